"""ctypes binding of include/crk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libcrk.so")

CRK_FP64, CRK_MIXED, CRK_MIXED_ADAPT = 0, 1, 2
STATUS = {0: "CRK_OK", 1: "CRK_WARN_SINGULAR", 2: "CRK_WARN_NOT_CONVERGED",
          -1: "CRK_ERR_INVALID_ARG", -2: "CRK_ERR_NONFINITE", -3: "CRK_ERR_SUPPORT",
          -4: "CRK_ERR_WORKSPACE", -5: "CRK_ERR_HIP", -6: "CRK_ERR_STATE",
          -7: "CRK_ERR_CAPACITY"}

# every symbol include/crk.h declares
EXPORTS = ("crk_params_default", "crk_create", "crk_destroy", "crk_last_error", "crk_build_cells",
           "crk_build_cells_batch", "crk_build_leaves",
           "crk_update_support", "crk_permute", "crk_moments", "crk_corrections",
           "crk_derivatives", "crk_hsolve", "crk_export_neighbors", "crk_set_lanes", "crk_set_wave_mapping", "crk_set_walk", "crk_set_hsolve",
           "crk_timing_enable", "crk_timing_only", "crk_timing_reset", "crk_timing_read", "crk_adaptive_rows",
           "crk_hnet_features", "crk_hnet_forward", "crk_hnet_train_step",
           "crk_hnet_train_step_noalloc", "crk_hnet_seed",
           "crk_hnet_targets", "crk_step", "crk_graph_capture", "crk_graph_replay",
           "crk_graph_destroy", "crk_set_timestep", "crk_timestep", "crk_compatible_energy",
           "crk_verlet_step", "crk_time_levels", "crk_workspace_bytes", "crk_workspace_estimate",
           "crk_version")

# members of crk_step_io, in order
STEP_INPUTS = ("x", "y", "z", "H", "v", "m", "u", "rho")
STEP_OUTPUTS = ("perm", "V", "m0", "m1", "m2", "gm0", "gm1", "gm2", "A", "B", "gA", "gB", "gradv",
                "dpdt", "dudt")


class StepIO(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in STEP_INPUTS + STEP_OUTPUTS]


VERLET_FIELDS = ("x", "y", "z", "H", "v", "m", "u", "rho", "dpdt", "dudt")

# values per particle of the arrays of crk_step_io and crk_verlet_io
STEP_COMPONENTS = dict(v=3, m1=3, m2=6, gm0=3, gm1=9, gm2=18, B=3, gA=3, gB=9, gradv=9, dpdt=3)


class VerletIO(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in VERLET_FIELDS]


class GraphStatus(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n_pairs", "n_singular", "n_fp64_rows",
                                         "n_touched_rows")] + \
               [(k, C.c_int32) for k in ("input_error", "overflow", "state_error", "reserved")]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CrkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("L", "gamma", "Cl", "Cq", "eps", "nh", "eta_crit",
                                          "eta_fold", "a", "adot", "kappa_max")] + \
               [("precision", C.c_int32), ("reserved", C.c_int32)]

    @classmethod
    def default(cls, nres: float = 64.0, **over) -> "Params":
        p = cls()
        st = lib().crk_params_default(C.byref(p), C.c_double(nres))
        if st != 0:
            raise CrkError(st, "crk_params_default")
        for k, v in over.items():
            setattr(p, k, v)
        return p

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def library_path() -> str:
    return _LIBPATH


def lib():
    """Load libcrk.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            raise RuntimeError(f"{_LIBPATH} is missing: build it with paper_2202_02840_amd/build.py")
        L = C.CDLL(_LIBPATH)
        p, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sigs = {
            "crk_params_default": ([p, d], i32),
            "crk_create": ([p, C.c_int, p], i32),
            "crk_destroy": ([p], None),
            "crk_last_error": ([p], C.c_char_p),
            "crk_build_cells": ([p, i64, p, p, p, p, p, d, p, p, p], i32),
            "crk_build_cells_batch": ([p, i32, p, i64, p, p, p, p, p, d, p, p, p], i32),
            "crk_build_leaves": ([p, i32, p, i64, p, p, p, p, p, i32, i32, p, p, p, p, i64], i32),
            "crk_update_support": ([p, p, p], i32),
            "crk_permute": ([p, p, p, i32, i32], i32),
            "crk_moments": ([p, p] + [p] * 8, i32),
            "crk_corrections": ([p, i64] + [p] * 11, i32),
            "crk_derivatives": ([p, p] + [p] * 12, i32),
            "crk_set_timestep": ([p, i32], i32),
            "crk_timestep": ([p, p, p, p, p, p, p, d, d, p, p, p, p], i32),
            "crk_compatible_energy": ([p, p] + [p] * 12 + [d, p], i32),
            "crk_verlet_step": ([p, i32, p, i64, p, p, d, d, i32, i32, p], i32),
            "crk_time_levels": ([p, p, p, p, d, d, i32, p, p, p, p], i32),
            "crk_workspace_bytes": ([p, p], i32),
            "crk_workspace_estimate": ([p, i64, i32, d, i32, i32, p], i32),
            "crk_hsolve": ([p, d, d, i32, p, p, p], i32),
            "crk_export_neighbors": ([p, i32, p, p, i64, p], i32),
            "crk_set_lanes": ([p, i32, i32, i32, i32], i32),
            "crk_set_wave_mapping": ([p, i32, i32, i32, i32], i32),
            "crk_set_walk": ([p, i32, i32, i32], i32),
            "crk_set_hsolve": ([p, i32, i32, i32, d], i32),
            "crk_timing_enable": ([p, i32], i32),
            "crk_timing_only": ([p, C.c_char_p], i32),
            "crk_timing_reset": ([p], i32),
            "crk_timing_read": ([p, C.c_char_p, p, p], i32),
            "crk_adaptive_rows": ([p, p, p], i32),
            "crk_hnet_features": ([p, d, p, p], i32),
            "crk_hnet_forward": ([p, p, p, i64, p], i32),
            "crk_hnet_train_step": ([p, p, p, p, i64, C.c_float, p, p, i64, p, p], i32),
            "crk_hnet_train_step_noalloc": ([p, p, p, p, i64, C.c_float, p, p, i64, p, p], i32),
            "crk_hnet_seed": ([p, p, d, p, p], i32),
            "crk_hnet_targets": ([p, i64, p, p, p], i32),
            "crk_step": ([p, i32, p, i64, p, p, d, p, p], i32),
            "crk_graph_capture": ([p, i32, p, i64, p, p, d, d], i32),
            "crk_graph_replay": ([p, p], i32),
            "crk_graph_destroy": ([p], i32),
            "crk_version": ([], C.c_char_p),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def version() -> str:
    return lib().crk_version().decode()


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("arrays must be device tensors")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous")
    return C.c_void_p(t.data_ptr())


def _f64(*ts):
    for t in ts:
        if t is not None and t.dtype != torch.float64:
            raise TypeError("boundary arrays are float64")


# parameters of the h-surrogate network 8 -> 64 -> 64 -> 1
HNET_PARAMS = 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def _arr(t, name: str, ncomp: int, n: int, dtype=torch.float64, optional: bool = False):
    """Checks one boundary array before it reaches a kernel: a contiguous
    device tensor of `dtype` holding ncomp * n values, shaped [n] (ncomp 1)
    or [ncomp, n] / [ncomp * n]. A wrongly sized array would otherwise be
    read or written out of bounds on the device."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    shape = tuple(t.shape)
    ok = n >= 0 and t.numel() == ncomp * n and (len(shape) == 1 or shape == (ncomp, n) or
                                                 (ncomp == 1 and shape == (1, n)))
    if not ok:
        want = f"[{n}]" if ncomp == 1 else f"[{ncomp}, {n}]"
        if n < 0:
            want = "a 1-D particle array"
        raise ValueError(f"{name}: expected shape {want}, got {list(shape)}")
    if not _on_device(t):
        raise ValueError(f"{name}: arrays must be device tensors")
    if not t.is_contiguous():
        raise ValueError(f"{name}: arrays must be contiguous")


def _on_device(t) -> bool:
    return t.is_cuda


WS_STEP, WS_HSOLVE, WS_HNET, WS_COMPAT, WS_VERLET, WS_GRAPH, WS_TIMESTEP, WS_LEAVES = \
    0, 1, 2, 4, 8, 16, 32, 64


def workspace_estimate(n: int, pairs_per_particle: float, precision: int, uses: int = 0,
                       nboxes: int = 1, ctx_handle=None) -> int:
    """crk_workspace_estimate: bytes, before any call (host only, no GPU needed)."""
    b = C.c_int64()
    st = lib().crk_workspace_estimate(ctx_handle, int(n), int(nboxes), C.c_double(pairs_per_particle),
                                      int(precision), int(uses), C.byref(b))
    if st != 0:
        raise CrkError(st, "crk_workspace_estimate: bad argument")
    return b.value


class Context:
    """One crk_ctx bound to a device and a HIP stream (torch's current stream
    by default)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the CRKSPH library runs on the device only")
        self.device = torch.device("cuda", device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = lib().crk_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise CrkError(st, "crk_create")
        self._h = h
        self.n = 0
        self.n_pairs = 0
        self.n_cells = 0
        self.perm = None

    def close(self):
        if getattr(self, "_h", None):
            lib().crk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str, allow_warn: bool = True) -> int:
        if st < 0 or (st > 0 and not allow_warn):
            raise CrkError(st, f"{what}: {lib().crk_last_error(self._h).decode()}")
        return st

    def _empty(self, *shape, dtype=torch.float64):
        return torch.empty(*shape, dtype=dtype, device=self.device)

    def _state_args(self, v, m, u, rho, V, corr: dict):
        n = self.n
        _arr(v, "v", 3, n)
        for k, t in (("m", m), ("u", u), ("V", V)):
            _arr(t, k, 1, n)
        _arr(rho, "rho", 1, n, optional=True)
        for k, nc in (("A", 1), ("B", 3), ("gA", 3), ("gB", 9)):
            _arr(corr.get(k), k, nc, n)

    def _hnet_args(self, theta, feat, m=None, v=None, target=None) -> int:
        nb = feat.shape[-1] if isinstance(feat, torch.Tensor) and feat.dim() == 2 else -1
        _arr(theta, "theta", 1, HNET_PARAMS, dtype=torch.float32)
        if isinstance(feat, torch.Tensor) and feat.dim() != 2:
            raise ValueError("feat: expected shape [8, nb]")
        _arr(feat, "feat", 8, nb, dtype=torch.float32)
        if target is not None or m is not None:
            _arr(m, "m", 1, HNET_PARAMS, dtype=torch.float32)
            _arr(v, "v", 1, HNET_PARAMS, dtype=torch.float32)
            _arr(target, "target", 1, nb, dtype=torch.float32)
        return nb

    # ---------------------------------------------------------------- S1
    def build_cells(self, x, y, z, H, params: Params, cell_size: float = 0.0):
        n = x.shape[0] if isinstance(x, torch.Tensor) and x.dim() == 1 else -1
        for k, t in (("x", x), ("y", y), ("z", z), ("H", H)):
            _arr(t, k, 1, n)
        perm = self._empty(n, dtype=torch.int32)
        npairs = C.c_int64()
        ncell = C.c_int32()
        st = lib().crk_build_cells(self._h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(H),
                                   C.byref(params), C.c_double(cell_size), _ptr(perm),
                                   C.byref(npairs), C.byref(ncell))
        self._check(st, "crk_build_cells")
        self.n, self.n_pairs, self.n_cells, self.perm = n, npairs.value, ncell.value, perm
        return perm, npairs.value

    def build_cells_batch(self, box_offsets, x, y, z, H, params: Params, cell_size: float = 0.0):
        """box_offsets: host sequence of nboxes+1 particle offsets (0 .. n)."""
        import numpy as np
        n = x.shape[0] if isinstance(x, torch.Tensor) and x.dim() == 1 else -1
        for k, t in (("x", x), ("y", y), ("z", z), ("H", H)):
            _arr(t, k, 1, n)
        off = np.ascontiguousarray(box_offsets, dtype=np.int64)
        if off.ndim != 1 or len(off) < 2:
            raise ValueError("box_offsets: expected nboxes + 1 offsets")
        perm = self._empty(n, dtype=torch.int32)
        npairs = C.c_int64()
        ncell = C.c_int32()
        st = lib().crk_build_cells_batch(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), n,
                                         _ptr(x), _ptr(y), _ptr(z), _ptr(H), C.byref(params),
                                         C.c_double(cell_size), _ptr(perm), C.byref(npairs),
                                         C.byref(ncell))
        self._check(st, "crk_build_cells_batch")
        self.n, self.n_pairs, self.n_cells, self.perm = n, npairs.value, ncell.value, perm
        return perm, npairs.value

    def build_leaves(self, x, y, z, H, params: Params, nppl: int = 256, bucket: int = 32,
                     box_offsets=None):
        """RCB leaf tiling (crk_build_leaves): returns (perm, n_pairs,
        leaf_offsets) with leaf_offsets a device int32 tensor [n_leaves+1]."""
        import numpy as np
        n = x.shape[0] if isinstance(x, torch.Tensor) and x.dim() == 1 else -1
        for k, t in (("x", x), ("y", y), ("z", z), ("H", H)):
            _arr(t, k, 1, n)
        off = np.ascontiguousarray([0, n] if box_offsets is None else box_offsets, dtype=np.int64)
        if off.ndim != 1 or len(off) < 2:
            raise ValueError("box_offsets: expected nboxes + 1 offsets")
        perm = self._empty(n, dtype=torch.int32)
        cap = n + len(off)
        loff = self._empty(cap, dtype=torch.int32)
        npairs = C.c_int64()
        nl = C.c_int32()
        st = lib().crk_build_leaves(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), n,
                                    _ptr(x), _ptr(y), _ptr(z), _ptr(H), C.byref(params),
                                    int(nppl), int(bucket), _ptr(perm), C.byref(npairs),
                                    C.byref(nl), _ptr(loff), cap)
        self._check(st, "crk_build_leaves")
        self.n, self.n_pairs, self.n_cells, self.perm = n, npairs.value, 0, perm
        return perm, npairs.value, loff[:nl.value + 1]

    def update_support(self, H_sorted):
        _arr(H_sorted, "H_sorted", 1, self.n)
        npairs = C.c_int64()
        self._check(lib().crk_update_support(self._h, _ptr(H_sorted), C.byref(npairs)),
                    "crk_update_support")
        self.n_pairs = npairs.value
        return npairs.value

    def permute(self, src, to_sorted: bool):
        ncomp = 1 if not isinstance(src, torch.Tensor) or src.dim() == 1 else src.shape[0]
        _arr(src, "src", ncomp, self.n)
        dst = torch.empty_like(src)
        self._check(lib().crk_permute(self._h, _ptr(src), _ptr(dst), ncomp, int(to_sorted)),
                    "crk_permute")
        return dst

    # ---------------------------------------------------------------- S2 + S4
    def moments(self, params: Params, want_moments: bool = True):
        n = self.n
        out = dict(nsum=self._empty(n), V=self._empty(n))
        if want_moments:
            out.update(m0=self._empty(n), m1=self._empty(3, n), m2=self._empty(6, n),
                       gm0=self._empty(3, n), gm1=self._empty(9, n), gm2=self._empty(18, n))
        keys = ("nsum", "V", "m0", "m1", "m2", "gm0", "gm1", "gm2")
        st = lib().crk_moments(self._h, C.byref(params), *[_ptr(out.get(k)) for k in keys])
        self._check(st, "crk_moments")
        return out

    # ---------------------------------------------------------------- S5
    def corrections(self, mom: dict, count_singular: bool = True):
        n = self.n
        for k, nc in (("m0", 1), ("m1", 3), ("m2", 6), ("gm0", 3), ("gm1", 9), ("gm2", 18)):
            _arr(mom.get(k), k, nc, n)
        out = dict(A=self._empty(n), B=self._empty(3, n), gA=self._empty(3, n),
                   gB=self._empty(9, n))
        ns = C.c_int64(-1)
        st = lib().crk_corrections(self._h, n, *[_ptr(mom[k]) for k in
                                                 ("m0", "m1", "m2", "gm0", "gm1", "gm2")],
                                   *[_ptr(out[k]) for k in ("A", "B", "gA", "gB")],
                                   C.byref(ns) if count_singular else None)
        self._check(st, "crk_corrections")
        out["n_singular"] = ns.value
        return out

    # ---------------------------------------------------------------- S6 + S7
    def derivatives(self, params: Params, v, m, u, rho, V, corr: dict):
        n = self.n
        self._state_args(v, m, u, rho, V, corr)
        out = dict(gradv=self._empty(9, n), dpdt=self._empty(3, n), dudt=self._empty(n))
        st = lib().crk_derivatives(self._h, C.byref(params), _ptr(v), _ptr(m), _ptr(u), _ptr(rho),
                                   _ptr(V), *[_ptr(corr[k]) for k in ("A", "B", "gA", "gB")],
                                   _ptr(out["gradv"]), _ptr(out["dpdt"]), _ptr(out["dudt"]))
        self._check(st, "crk_derivatives")
        return out

    def set_timestep(self, on: bool = True):
        self._check(lib().crk_set_timestep(self._h, int(bool(on))), "crk_set_timestep")

    def timestep(self, params: Params, u, m, rho, V, gradv, zeta: float = 4.0, c_cfl: float = 0.25):
        """Courant terms after a crk_derivatives call made with set_timestep
        on (sorted order): dict of vsig, csq, vmax, dt_hyd."""
        n = self.n
        for k, t in (("u", u), ("m", m), ("V", V)):
            _arr(t, k, 1, n)
        _arr(rho, "rho", 1, n, optional=True)
        _arr(gradv, "gradv", 9, n)
        out = dict(vsig=self._empty(n), csq=self._empty(n), vmax=self._empty(n), dt_hyd=self._empty(n))
        st = lib().crk_timestep(self._h, C.byref(params), _ptr(u), _ptr(m), _ptr(rho), _ptr(V),
                                _ptr(gradv), C.c_double(zeta), C.c_double(c_cfl), _ptr(out["vsig"]),
                                _ptr(out["csq"]), _ptr(out["vmax"]), _ptr(out["dt_hyd"]))
        self._check(st, "crk_timestep")
        return out

    def compatible_energy(self, params: Params, v, m, u, rho, V, corr: dict, gradv, dpdt,
                          dt: float, pk=None):
        """Delta u of the compatible energy update over dt (sorted order),
        from the state and outputs of the preceding derivative call; pk:
        optional kick-start momenta [3, n] (sorted)."""
        n = self.n
        self._state_args(v, m, u, rho, V, corr)
        _arr(gradv, "gradv", 9, n)
        _arr(dpdt, "dpdt", 3, n)
        _arr(pk, "pk", 3, n, optional=True)
        du = self._empty(self.n)
        st = lib().crk_compatible_energy(self._h, C.byref(params), _ptr(v), _ptr(m), _ptr(u),
                                         _ptr(rho), _ptr(V),
                                         *[_ptr(corr[k]) for k in ("A", "B", "gA", "gB")],
                                         _ptr(gradv), _ptr(dpdt), _ptr(pk), C.c_double(dt),
                                         _ptr(du))
        self._check(st, "crk_compatible_energy")
        return du

    def workspace_estimate(self, n: int, pairs_per_particle: float, precision: int, uses: int = 0,
                           nboxes: int = 1) -> int:
        """Upper bound on the workspace bytes for calls on n particles
        (crk_workspace_estimate with this context's tuning)."""
        return workspace_estimate(n, pairs_per_particle, precision, uses, nboxes, self._h)

    def workspace_bytes(self) -> int:
        """Device bytes the context's workspace holds now."""
        b = C.c_int64()
        self._check(lib().crk_workspace_bytes(self._h, C.byref(b)), "crk_workspace_bytes")
        return b.value

    def time_levels(self, params: Params, dt_hyd, dpdt, r_soft: float, dt_sub: float,
                    l_max: int = 20):
        """Time-step levels (crk_time_levels), sorted order: dict of dt_acc,
        dt_min, level (int32) and n_over."""
        n = self.n
        _arr(dt_hyd, "dt_hyd", 1, n)
        _arr(dpdt, "dpdt", 3, n)
        out = dict(dt_acc=self._empty(n), dt_min=self._empty(n),
                   level=self._empty(n, dtype=torch.int32))
        nov = C.c_int64()
        st = lib().crk_time_levels(self._h, C.byref(params), _ptr(dt_hyd), _ptr(dpdt),
                                   C.c_double(r_soft), C.c_double(dt_sub), int(l_max),
                                   _ptr(out["dt_acc"]), _ptr(out["dt_min"]), _ptr(out["level"]),
                                   C.byref(nov))
        self._check(st, "crk_time_levels")
        out["n_over"] = nov.value
        return out

    # ---------------------------------------------------------------- whole step / S10 graph
    def step_buffers(self, dev: dict) -> dict:
        """Inputs of `dev` (original order) plus freshly allocated outputs."""
        n = dev["x"].shape[0]
        e = self._empty
        io = {k: dev.get(k) for k in STEP_INPUTS}
        io.update(perm=e(n, dtype=torch.int32), V=e(n), m0=e(n), m1=e(3, n), m2=e(6, n),
                  gm0=e(3, n), gm1=e(9, n), gm2=e(18, n), A=e(n), B=e(3, n), gA=e(3, n),
                  gB=e(9, n), gradv=e(9, n), dpdt=e(3, n), dudt=e(n))
        return io

    def _io(self, io: dict):
        x = io.get("x")
        n = x.shape[0] if isinstance(x, torch.Tensor) and x.dim() == 1 else -1
        for k in STEP_INPUTS + STEP_OUTPUTS:
            _arr(io.get(k), k, STEP_COMPONENTS.get(k, 1), n,
                 dtype=torch.int32 if k == "perm" else torch.float64, optional=(k == "rho"))
        s = StepIO()
        for k in STEP_INPUTS + STEP_OUTPUTS:
            setattr(s, k, None if io.get(k) is None else io[k].data_ptr())
            if io.get(k) is not None:
                _ptr(io[k])
        return s

    def step(self, io: dict, params: Params, box_offsets=None, cell_size: float = 0.0):
        """crk_step on the buffers of `io` (see step_buffers); returns
        (n_pairs, n_singular)."""
        import numpy as np
        n = io["x"].shape[0]
        off = np.ascontiguousarray([0, n] if box_offsets is None else box_offsets, dtype=np.int64)
        s = self._io(io)
        npairs, ns = C.c_int64(), C.c_int64()
        st = lib().crk_step(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), n, C.byref(s),
                            C.byref(params), C.c_double(cell_size), C.byref(npairs), C.byref(ns))
        self._check(st, "crk_step")
        self.n, self.n_pairs, self.perm = n, npairs.value, io["perm"]
        return npairs.value, ns.value

    def verlet_step(self, state: dict, params: Params, dt: float, start_eval: bool = False,
                    box_offsets=None, cell_size: float = 0.0, energy: str = "eng") -> int:
        """One velocity-Verlet step (crk_verlet_step) on the device arrays of
        `state` (x, y, z, H, v, m, u, optional rho, dpdt, dudt; the caller's
        order), advanced in place; energy "eng" (du/dt of eq. eng) or
        "compat" (compatible update per half kick). Returns the end
        evaluation's pair count."""
        mode = {"eng": 0, "compat": 1}[energy]
        import numpy as np
        x = state.get("x")
        n = x.shape[0] if isinstance(x, torch.Tensor) and x.dim() == 1 else -1
        for k in VERLET_FIELDS:
            _arr(state.get(k), k, STEP_COMPONENTS.get(k, 1), n, optional=(k == "rho"))
        off = np.ascontiguousarray([0, n] if box_offsets is None else box_offsets, dtype=np.int64)
        s = VerletIO(*[_ptr(state.get(k)) for k in VERLET_FIELDS])
        npairs = C.c_int64()
        st = lib().crk_verlet_step(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), n,
                                   C.byref(s), C.byref(params), C.c_double(cell_size),
                                   C.c_double(dt), int(bool(start_eval)), mode, C.byref(npairs))
        self._check(st, "crk_verlet_step")
        self.n, self.n_pairs = n, npairs.value
        return npairs.value

    def graph_capture(self, io: dict, params: Params, box_offsets=None, cell_size: float = 0.0,
                      headroom: float = 0.25):
        """Record the step on the buffers of `io` as a graph (the buffers are
        kept alive with the graph); the outputs hold the step's results."""
        import numpy as np
        n = io["x"].shape[0]
        off = np.ascontiguousarray([0, n] if box_offsets is None else box_offsets, dtype=np.int64)
        s = self._io(io)
        st = lib().crk_graph_capture(self._h, len(off) - 1, off.ctypes.data_as(C.c_void_p), n,
                                     C.byref(s), C.byref(params), C.c_double(cell_size),
                                     C.c_double(headroom))
        self._check(st, "crk_graph_capture")
        self._graph_io = io
        self.n, self.perm = n, io["perm"]

    def graph_replay(self, status: bool = True, check: bool = True):
        """Replay the recorded step; with status, wait and return (status
        code, status dict). check raises on an error code."""
        if not status:
            self._check(lib().crk_graph_replay(self._h, None), "crk_graph_replay")
            return 0, None
        gs = GraphStatus()
        st = lib().crk_graph_replay(self._h, C.byref(gs))
        if check:
            self._check(st, "crk_graph_replay")
        self.n_pairs = gs.n_pairs
        return st, gs.as_dict()

    def graph_destroy(self):
        self._check(lib().crk_graph_destroy(self._h), "crk_graph_destroy")
        self._graph_io = None

    # ---------------------------------------------------------------- S3
    def hsolve(self, Nres: float, H_sorted, tol: float = 1e-7, max_iter: int = 100):
        _arr(H_sorted, "H_sorted", 1, self.n)
        Hio = H_sorted.clone()
        iters = self._empty(self.n, dtype=torch.int32)
        nun = C.c_int64()
        st = lib().crk_hsolve(self._h, C.c_double(Nres), C.c_double(tol), max_iter, _ptr(Hio),
                              _ptr(iters), C.byref(nun))
        self._check(st, "crk_hsolve")
        return Hio, iters, nun.value

    # ---------------------------------------------------------------- checks / tuning
    def export_neighbors(self, which: int):
        n = self.n
        off = self._empty(n + 1, dtype=torch.int64)
        tot = C.c_int64()
        self._check(lib().crk_export_neighbors(self._h, which, _ptr(off), None, 0, C.byref(tot)),
                    "crk_export_neighbors")
        idx = self._empty(max(tot.value, 1), dtype=torch.int32)
        self._check(lib().crk_export_neighbors(self._h, which, _ptr(off), _ptr(idx), tot.value,
                                               C.byref(tot)), "crk_export_neighbors")
        return off, idx[:tot.value]

    def timing(self, on: bool):
        self._check(lib().crk_timing_enable(self._h, int(on)), "crk_timing_enable")

    def timing_only(self, kernel=None):
        """Time only this kernel name while timing is on (None: every kernel)."""
        self._check(lib().crk_timing_only(self._h, kernel.encode() if kernel else None),
                    "crk_timing_only")

    def timing_reset(self):
        self._check(lib().crk_timing_reset(self._h), "crk_timing_reset")

    def timing_read(self, kernel: str):
        """(summed event time in ms, launches) of one kernel name."""
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(lib().crk_timing_read(self._h, kernel.encode(), C.byref(ms), C.byref(cnt)),
                    "crk_timing_read")
        return ms.value, cnt.value

    def adaptive_rows(self):
        """(FP64 rows, touched rows) of the last adaptive derivative pass."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().crk_adaptive_rows(self._h, C.byref(a), C.byref(b)), "crk_adaptive_rows")
        return a.value, b.value

    # ---------------------------------------------------------------- S9
    def hnet_features(self, Nres: float, H_sorted):
        _arr(H_sorted, "H_sorted", 1, self.n)
        feat = self._empty(8, self.n, dtype=torch.float32)
        self._check(lib().crk_hnet_features(self._h, C.c_double(Nres), _ptr(H_sorted), _ptr(feat)),
                    "crk_hnet_features")
        return feat

    def hnet_forward(self, theta, feat):
        nb = self._hnet_args(theta, feat)
        y = self._empty(nb, dtype=torch.float32)
        self._check(lib().crk_hnet_forward(self._h, _ptr(theta), _ptr(feat), nb, _ptr(y)),
                    "crk_hnet_forward")
        return y

    def hnet_train_step(self, theta, m, v, step: int, lr: float, feat, target, want_grad=False,
                        want_loss=False):
        """One Adam step in place on theta/m/v (lr > 0); returns (grad, loss)."""
        nb = self._hnet_args(theta, feat, m, v, target)
        grad = self._empty(theta.shape[0], dtype=torch.float32) if want_grad else None
        loss = C.c_float()
        self._check(lib().crk_hnet_train_step(self._h, _ptr(theta), _ptr(m), _ptr(v), step,
                                              C.c_float(lr), _ptr(feat), _ptr(target), nb,
                                              _ptr(grad), C.byref(loss) if want_loss else None),
                    "crk_hnet_train_step")
        return grad, (loss.value if want_loss else None)

    def hnet_train_step_noalloc(self, theta, m, v, step: int, lr: float, feat, target,
                                grad=None, loss=None):
        """crk_hnet_train_step_noalloc: one Adam step in place on theta/m/v
        (lr > 0) with the static scratch (at most 8192 samples); grad
        (float32 [4801]) and loss (float32 [1]) are optional device outputs
        written on the stream."""
        nb = self._hnet_args(theta, feat, m, v, target)
        _arr(grad, "grad", 1, HNET_PARAMS, dtype=torch.float32, optional=True)
        _arr(loss, "loss", 1, 1, dtype=torch.float32, optional=True)
        self._check(lib().crk_hnet_train_step_noalloc(self._h, _ptr(theta), _ptr(m), _ptr(v), step,
                                                      C.c_float(lr), _ptr(feat), _ptr(target), nb,
                                                      _ptr(grad), _ptr(loss)),
                    "crk_hnet_train_step_noalloc")

    def hnet_seed(self, theta, Nres: float, H_prev_sorted):
        _arr(theta, "theta", 1, HNET_PARAMS, dtype=torch.float32)
        _arr(H_prev_sorted, "H_prev_sorted", 1, self.n)
        out = torch.empty_like(H_prev_sorted)
        self._check(lib().crk_hnet_seed(self._h, _ptr(theta), C.c_double(Nres),
                                        _ptr(H_prev_sorted), _ptr(out)), "crk_hnet_seed")
        return out

    def hnet_targets(self, H_prev, H_conv):
        nb = H_prev.shape[0] if isinstance(H_prev, torch.Tensor) and H_prev.dim() == 1 else -1
        _arr(H_prev, "H_prev", 1, nb)
        _arr(H_conv, "H_conv", 1, nb)
        t = self._empty(H_prev.shape[0], dtype=torch.float32)
        self._check(lib().crk_hnet_targets(self._h, H_prev.shape[0], _ptr(H_prev), _ptr(H_conv),
                                           _ptr(t)), "crk_hnet_targets")
        return t

    def set_hsolve(self, lanes: int = 0, round: int = 0, cap: int = 0, factor: float = 0.0):
        self._check(lib().crk_set_hsolve(self._h, lanes, round, cap, C.c_double(factor)),
                    "crk_set_hsolve")

    def set_walk(self, lanes: int = 0, cap: int = 0, level_shift: int = -1):
        self._check(lib().crk_set_walk(self._h, lanes, cap, level_shift), "crk_set_walk")

    def set_wave_mapping(self, vol: int = -1, mom: int = -1, grad: int = -1, deriv: int = -1):
        """Volume / moment / velocity-gradient / derivative passes: 4, 8, 16
        or 32 particles per wavefront with lanes split by row length, 0 for
        set_lanes' lanes per particle, -1 to keep."""
        self._check(lib().crk_set_wave_mapping(self._h, int(vol), int(mom), int(grad), int(deriv)),
                    "crk_set_wave_mapping")

    def set_lanes(self, vol: int = 0, mom: int = 0, grad: int = 0, der: int = 0):
        self._check(lib().crk_set_lanes(self._h, vol, mom, grad, der), "crk_set_lanes")
