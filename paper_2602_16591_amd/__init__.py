"""pswfe: PSWF fast Ewald summation (long-range part) on AMD MI355X.

Thin ctypes binding of the C-ABI declared in ``include/pswfe.h``; every step of the
computation runs in the HIP library ``_lib/libpswfe.so``. PyTorch supplies device memory and
streams only. There is no CPU fallback: without the built library, or with tensors that are
not on a HIP device, calls raise.

Method: Bostrom, Tornberg, af Klinteberg, arXiv 2602.16591 (Alg. 2 fast Fourier-space sum,
Sec. 4 PSWF mollifier and window, Alg. 3 parameter selection).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpswfe.so")

OK, E_ARG, E_EPS_RANGE, E_GRID, E_ALLOC, E_HIP, E_CAPACITY, E_PREC, E_NONNEUTRAL, E_NONFINITE = range(10)
TOL_REL, TOL_ABS = 0, 1
FP32, FP64, FP32_ARITH = 0, 1, 2
PRECISIONS = {"fp32": FP32, "fp64": FP64, "fp32_arith": FP32_ARITH}
VEC_GRAD, TOTAL, CHECK_INPUT = 1, 2, 4


class PswfeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib().pswfe_status_str(status).decode()} (status {status})")


class CParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("eps", ctypes.c_double), ("rc", ctypes.c_double),
                ("cs", ctypes.c_double), ("cw", ctypes.c_double), ("alpha", ctypes.c_double),
                ("h", ctypes.c_double), ("lambda0_s", ctypes.c_double), ("cs_alg", ctypes.c_double),
                ("cw_alg", ctypes.c_double), ("alpha_alg", ctypes.c_double), ("m", ctypes.c_int32),
                ("P", ctypes.c_int32), ("tol_mode", ctypes.c_int32), ("split", ctypes.c_int32),
                ("window", ctypes.c_int32), ("reserved", ctypes.c_int32), ("cg", ctypes.c_double),
                ("Ly", ctypes.c_double), ("Lz", ctypes.c_double), ("my", ctypes.c_int32), ("mz", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


# name -> (restype, argtypes); every symbol declared in include/pswfe.h
_vp, _i64, _i32, _d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_PPlan = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "pswfe_choose_params": (ctypes.c_int, [_d, _d, _d, _i32, _i64, _d, _i32, ctypes.POINTER(CParams)]),
    "pswfe_choose_params_box": (ctypes.c_int, [_d, _d, _d, _d, _d, _i32, _i64, _d, _i32, ctypes.POINTER(CParams)]),
    "pswfe_oversample_params": (ctypes.c_int, [ctypes.POINTER(CParams), _d, ctypes.POINTER(CParams)]),
    "pswfe_variant_params": (ctypes.c_int, [_i32, _i32, _d, _d, _d, _i32, _i32, _d, _d, ctypes.POINTER(CParams)]),
    "pswfe_plan_create": (ctypes.c_int, [ctypes.POINTER(CParams), _i32, _i64, _PPlan]),
    "pswfe_plan_create_tiled": (ctypes.c_int, [ctypes.POINTER(CParams), _i32, _i64, _i32, _PPlan]),
    "pswfe_plan_tile": (ctypes.c_int32, [_vp]),
    "pswfe_plan_destroy": (ctypes.c_int, [_vp]),
    "pswfe_compute": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_compute_grad": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_compute_noalloc": (ctypes.c_int, [ctypes.POINTER(CParams), _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_spread": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "pswfe_transform": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pswfe_interpolate": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_plan_params": (ctypes.c_int, [_vp, ctypes.POINTER(CParams)]),
    "pswfe_batch_plan_create": (ctypes.c_int, [_i32, ctypes.POINTER(CParams), ctypes.POINTER(ctypes.c_int64), _i32,
                                               ctypes.POINTER(ctypes.c_int32), _PPlan]),
    "pswfe_batch_compute": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_batch_compute_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pswfe_plan_num_systems": (ctypes.c_int32, [_vp]),
    "pswfe_compute_ex": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "pswfe_batch_compute_ex": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "pswfe_local": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "pswfe_host_local": (ctypes.c_int, [ctypes.POINTER(CParams), _i64, _vp, _vp, _vp, _vp]),
    "pswfe_plan_system": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(CParams), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "pswfe_host_pswf": (ctypes.c_int, [_d, _d, _vp, _vp, _vp, _vp]),
    "pswfe_host_tables": (ctypes.c_int, [ctypes.POINTER(CParams), _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "pswfe_timing_enable": (ctypes.c_int, [_vp, _i32, _i32]),
    "pswfe_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "pswfe_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "pswfe_version": (ctypes.c_char_p, []),
}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2602_16591_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(status: int, where: str):
    if status != OK:
        raise PswfeError(status, where)


def version() -> str:
    return _lib().pswfe_version().decode()


def choose_params(eps: float, L: float, *, rc: float = 0.0, m: int = 0, n: int = 0, q_l2: float = 0.0,
                  tol_mode: int | str = TOL_REL) -> CParams:
    """Alg. 3 parameters (host only)."""
    mode = {"rel": TOL_REL, "abs": TOL_ABS}.get(tol_mode, tol_mode)
    out = CParams()
    _check(_lib().pswfe_choose_params(float(eps), float(L), float(rc), int(m), int(n), float(q_l2), int(mode),
                                      ctypes.byref(out)), "pswfe_choose_params")
    return out


def choose_params_box(eps: float, box, *, rc: float = 0.0, m: int = 0, n: int = 0, q_l2: float = 0.0,
                      tol_mode: int | str = TOL_REL) -> CParams:
    """Alg. 3 for a cuboid box (Lx, Ly, Lz) (host only); m is the grid size along the shortest side."""
    Lx, Ly, Lz = (float(v) for v in box)
    mode = {"rel": TOL_REL, "abs": TOL_ABS}.get(tol_mode, tol_mode)
    out = CParams()
    _check(_lib().pswfe_choose_params_box(float(eps), Lx, Ly, Lz, float(rc), int(m), int(n), float(q_l2), int(mode),
                                          ctypes.byref(out)), "pswfe_choose_params_box")
    return out


def oversample_params(params: CParams, sigma: float) -> CParams:
    """PSWF/PSWF parameters on a grid oversampled by sigma, with the smaller support it allows
    (host only)."""
    out = CParams()
    _check(_lib().pswfe_oversample_params(ctypes.byref(params), float(sigma), ctypes.byref(out)),
           "pswfe_oversample_params")
    return out


SPLITS = {"pswf": 0, "gauss": 1}
WINDOWS = {"pswf": 0, "gauss": 1, "bspline": 2}


def variant_params(split: int | str, window: int | str, L: float, rc: float, cs: float, m: int, P: int, *,
                   cg: float = 0.0, eps: float = 1e-6) -> CParams:
    """Parameters of a comparison configuration (split "pswf" | "gauss", window "pswf" | "gauss" |
    "bspline") with a given grid size m and support P (host only)."""
    out = CParams()
    _check(_lib().pswfe_variant_params(int(SPLITS.get(split, split)), int(WINDOWS.get(window, window)), float(L),
                                       float(rc), float(cs), int(m), int(P), float(cg), float(eps),
                                       ctypes.byref(out)), "pswfe_variant_params")
    return out


def host_pswf(c: float, x: float):
    """(psi_0^c(x), psi_0^c'(x), lambda_0(c), chi_0(c)) from the library's float64 host code."""
    out = (ctypes.c_double * 4)()
    a = ctypes.addressof(out)
    _check(_lib().pswfe_host_pswf(float(c), float(x), a, a + 8, a + 16, a + 24), "pswfe_host_pswf")
    return tuple(out)


def host_tables(params: CParams, prec: int | str = FP32):
    """The plan's float64 host tables: dict(tm, w, coef (P, deg+1), deg, fit_err, fit_err_deriv, self_coef)."""
    import numpy as np
    prec = PRECISIONS.get(prec, prec)
    m, P = params.m, params.P
    tm = np.zeros(3 * (m // 2) ** 2 + 1)
    w = np.zeros(m // 2 + 1)
    coef = np.zeros(P * 40)
    info = np.zeros(4)
    _check(_lib().pswfe_host_tables(ctypes.byref(params), int(prec), tm.ctypes.data, tm.size, w.ctypes.data, w.size,
                                    coef.ctypes.data, coef.size, info.ctypes.data), "pswfe_host_tables")
    deg = int(info[0])
    return dict(tm=tm, w=w, coef=coef[:P * (deg + 1)].reshape(P, deg + 1), deg=deg, fit_err=info[1],
                fit_err_deriv=info[2], self_coef=info[3])


def host_local(params: CParams, r):
    """The real-space residual the kernels evaluate, on the host: (R(r), R'(r)/r, info) for
    radii r (float64 array); info = (degree, fit error, K)."""
    import numpy as np
    r = np.ascontiguousarray(r, dtype=np.float64)
    R, dRr, info = np.zeros_like(r), np.zeros_like(r), np.zeros(3)
    _check(_lib().pswfe_host_local(ctypes.byref(params), r.size, r.ctypes.data, R.ctypes.data, dRr.ctypes.data,
                                   info.ctypes.data), "pswfe_host_local")
    return R, dRr, dict(deg=int(info[0]), fit_err=info[1], K=info[2])


def _ptr(t, dtype, shape_tail, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} must have shape (n, {', '.join(map(str, shape_tail))})")
    return t.data_ptr()


def _expect_shapes(**named):
    """Raises ValueError unless every tensor given (name=(tensor, shape)) has exactly that shape:
    the kernels index every array up to n (or the number of systems), so a short buffer would be
    read or written out of bounds. Checked before any pointer is passed to the library."""
    for name, (t, shape) in named.items():
        if t is None:
            continue
        got = tuple(getattr(t, "shape", ()))
        if got != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {got}")


def _out(spec, shape, dtype, device):
    """An output buffer: the tensor passed, a new tensor (True) or None (False/None)."""
    import torch
    if isinstance(spec, torch.Tensor):
        return spec
    return torch.empty(shape, dtype=dtype, device=device) if spec else None


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _prec(prec):
    p = PRECISIONS.get(prec, prec)
    if p not in (FP32, FP64, FP32_ARITH):
        raise ValueError(f"unknown precision {prec!r}")
    return p


class _PlanBase:
    _h = ctypes.c_void_p()

    def _init_common(self, prec):
        import torch
        self.prec = _prec(prec)
        self.dtype = torch.float64 if self.prec == FP64 else torch.float32
        self._h = ctypes.c_void_p()

    def system(self, s: int):
        """(effective parameters, first packed row, particle count, tile edge) of system s."""
        p, off, cnt, tile = CParams(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(_lib().pswfe_plan_system(self._h, int(s), ctypes.byref(p), ctypes.byref(off), ctypes.byref(cnt),
                                        ctypes.byref(tile)), "pswfe_plan_system")
        return p, off.value, cnt.value, tile.value

    def close(self):
        if self._h:
            _lib().pswfe_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = {"bin": 0, "spread": 1, "fft_x": 2, "fft_y": 3, "fft_z_scale": 4, "ifft_y": 5, "ifft_x": 6,
              "gather": 7, "all": 8, "local": 9}

    def timing_enable(self, stage: str | int | None, max_calls: int = 4096):
        """Record HIP events around one pipeline stage of the following calls (None: off)."""
        st = -1 if stage is None else self.STAGES.get(stage, stage)
        _check(_lib().pswfe_timing_enable(self._h, int(st), int(max_calls)), "pswfe_timing_enable")

    def timing_read(self):
        """(total milliseconds, number of timed calls) since enable or the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib().pswfe_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)), "pswfe_timing_read")
        return ms.value, n.value

    def graph(self, pos, q, **kw):
        """This plan's compute call on (pos, q) captured into a HIP graph; see CapturedCompute."""
        from .graph import CapturedCompute
        return CapturedCompute(self, pos, q, **kw)


class Plan(_PlanBase):
    """Device plan for one parameter set, precision and maximum particle count."""

    def __init__(self, params: CParams, prec: int | str = FP32, n_max: int = 0, tile: int = 0):
        self._init_common(prec)
        self.n_max = int(n_max)
        _check(_lib().pswfe_plan_create_tiled(ctypes.byref(params), int(self.prec), self.n_max, int(tile),
                                              ctypes.byref(self._h)), "pswfe_plan_create_tiled")
        self.tile = int(_lib().pswfe_plan_tile(self._h))
        p = CParams()
        _check(_lib().pswfe_plan_params(self._h, ctypes.byref(p)), "pswfe_plan_params")
        self.params = p

    @property
    def m(self) -> int:
        return self.params.m

    @property
    def grid_shape(self):
        """(mz, my, m): the grids' layout, x fastest (a cube: (m, m, m))."""
        p = self.params
        return (p.mz or p.m, p.my or p.m, p.m)

    def _n(self, pos):
        n = int(pos.shape[0])
        if n > self.n_max:
            raise ValueError(f"n = {n} exceeds the plan's n_max = {self.n_max}")
        return n

    def compute(self, pos, q, *, phi=True, force=True, energy=True, grad=False, total=False, check=False,
                stream=None):
        """phi_far + phi_self, forces -q grad phi_far (or grad phi_far with grad=True), energy;
        with total=True the real-space residual is included (the full Ewald sum). check=True
        first checks on the device that the charges sum to zero and every input is finite
        (PswfeError E_NONNEUTRAL / E_NONFINITE; synchronises the stream, not capturable).

        Returns (phi, vec, energy) with None for outputs not requested; outputs are new tensors
        unless tensors are passed in place of True."""
        import torch
        n = self._n(pos)
        phi_t = _out(phi, (n,), self.dtype, pos.device)
        vec_t = _out(force if not grad else grad, (n, 3), self.dtype, pos.device)
        e_t = _out(energy, (1,), torch.float64, pos.device)
        _expect_shapes(pos=(pos, (n, 3)), q=(q, (n,)), phi=(phi_t, (n,)), force=(vec_t, (n, 3)), energy=(e_t, (1,)))
        flags = (VEC_GRAD if grad else 0) | (TOTAL if total else 0) | (CHECK_INPUT if check else 0)
        _check(_lib().pswfe_compute_ex(self._h, n, _ptr(pos, self.dtype, (3,), "pos"), _ptr(q, self.dtype, None, "q"),
                                       _ptr(phi_t, self.dtype, None, "phi"), _ptr(vec_t, self.dtype, (3,), "force"),
                                       _ptr(e_t, torch.float64, None, "energy"), flags, _stream_ptr(stream)),
               "pswfe_compute_ex")
        return phi_t, vec_t, e_t

    def local(self, pos, q, *, phi=True, force=True, energy=True, grad=False, stream=None):
        """The real-space residual alone: (phi_local, force or grad, energy)."""
        import torch
        n = self._n(pos)
        phi_t = _out(phi, (n,), self.dtype, pos.device)
        vec_t = _out(force if not grad else grad, (n, 3), self.dtype, pos.device)
        e_t = _out(energy, (1,), torch.float64, pos.device)
        _expect_shapes(pos=(pos, (n, 3)), q=(q, (n,)), phi=(phi_t, (n,)), force=(vec_t, (n, 3)), energy=(e_t, (1,)))
        _check(_lib().pswfe_local(self._h, n, _ptr(pos, self.dtype, (3,), "pos"), _ptr(q, self.dtype, None, "q"),
                                  _ptr(phi_t, self.dtype, None, "phi"), _ptr(vec_t, self.dtype, (3,), "force"),
                                  _ptr(e_t, torch.float64, None, "energy"), VEC_GRAD if grad else 0,
                                  _stream_ptr(stream)), "pswfe_local")
        return phi_t, vec_t, e_t

    def spread(self, pos, q, grid=None, stream=None):
        import torch
        n = self._n(pos)
        grid = torch.empty(self.grid_shape, dtype=self.dtype, device=pos.device) if grid is None else grid
        _expect_shapes(pos=(pos, (n, 3)), q=(q, (n,)))
        if grid.numel() != math.prod(self.grid_shape):
            raise ValueError(f"grid must have {math.prod(self.grid_shape)} entries")
        _check(_lib().pswfe_spread(self._h, n, _ptr(pos, self.dtype, (3,), "pos"), _ptr(q, self.dtype, None, "q"),
                                   _ptr(grid, self.dtype, None, "grid"), _stream_ptr(stream)), "pswfe_spread")
        return grid

    def transform(self, grid_in, grid_out=None, stream=None):
        import torch
        grid_out = torch.empty_like(grid_in) if grid_out is None else grid_out
        size = math.prod(self.grid_shape)
        if grid_in.numel() != size or grid_out.numel() != size:
            raise ValueError(f"grids must have {size} entries")
        _check(_lib().pswfe_transform(self._h, _ptr(grid_in, self.dtype, None, "grid_in"),
                                      _ptr(grid_out, self.dtype, None, "grid_out"), _stream_ptr(stream)),
               "pswfe_transform")
        return grid_out

    def interpolate(self, pos, grid, stream=None):
        import torch
        n = self._n(pos)
        _expect_shapes(pos=(pos, (n, 3)))
        if grid.numel() != math.prod(self.grid_shape):
            raise ValueError(f"grid must have {math.prod(self.grid_shape)} entries")
        phi = torch.empty(n, dtype=self.dtype, device=pos.device)
        g = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        _check(_lib().pswfe_interpolate(self._h, n, _ptr(pos, self.dtype, (3,), "pos"),
                                        _ptr(grid, self.dtype, None, "grid"), _ptr(phi, self.dtype, None, "phi"),
                                        _ptr(g, self.dtype, (3,), "grad"), _stream_ptr(stream)), "pswfe_interpolate")
        return phi, g


class BatchPlan(_PlanBase):
    """Device plan for a batch of independent systems (own box, parameters and particle count
    each), run by one launch per pipeline stage. Particle arrays are packed: system s owns rows
    offsets[s] .. offsets[s] + counts[s] - 1."""

    def __init__(self, params, counts, prec: int | str = FP32, tiles=None):
        self._init_common(prec)
        params = list(params)
        counts = [int(c) for c in counts]
        ns = len(params)
        if ns == 0 or len(counts) != ns or (tiles is not None and len(tiles) != ns):
            raise ValueError("params, counts (and tiles) must be non-empty and of equal length")
        arr = (CParams * ns)(*params)
        cnt = (ctypes.c_int64 * ns)(*counts)
        tl = (ctypes.c_int32 * ns)(*[int(t) for t in tiles]) if tiles is not None else None
        _check(_lib().pswfe_batch_plan_create(ns, arr, cnt, int(self.prec), tl, ctypes.byref(self._h)),
               "pswfe_batch_plan_create")
        self.nsys = int(_lib().pswfe_plan_num_systems(self._h))
        info = [self.system(s) for s in range(self.nsys)]
        self.params = [i[0] for i in info]
        self.offsets = [i[1] for i in info]
        self.counts = [i[2] for i in info]
        self.tiles = [i[3] for i in info]
        self.n_total = sum(self.counts)
        self.P = self.params[0].P

    def compute(self, pos, q, *, phi=True, force=True, energy=True, grad=False, total=False, check=False,
                stream=None):
        """Every system at once. pos (N, 3), q (N,) packed; returns (phi (N,), vec (N, 3),
        energy (nsys,) float64) with None for outputs not requested (or the tensors passed);
        total=True includes the real-space residual; check=True as for Plan.compute, per system."""
        import torch
        n = self.n_total
        _expect_shapes(pos=(pos, (n, 3)), q=(q, (n,)))
        phi_t = _out(phi, (n,), self.dtype, pos.device)
        vec_t = _out(force if not grad else grad, (n, 3), self.dtype, pos.device)
        e_t = _out(energy, (self.nsys,), torch.float64, pos.device)
        _expect_shapes(phi=(phi_t, (n,)), force=(vec_t, (n, 3)), energy=(e_t, (self.nsys,)))
        flags = (VEC_GRAD if grad else 0) | (TOTAL if total else 0) | (CHECK_INPUT if check else 0)
        _check(_lib().pswfe_batch_compute_ex(self._h, _ptr(pos, self.dtype, (3,), "pos"),
                                             _ptr(q, self.dtype, None, "q"), _ptr(phi_t, self.dtype, None, "phi"),
                                             _ptr(vec_t, self.dtype, (3,), "force"),
                                             _ptr(e_t, torch.float64, None, "energy"), flags, _stream_ptr(stream)),
               "pswfe_batch_compute_ex")
        return phi_t, vec_t, e_t

    def split(self, a):
        """Per-system views of a packed array."""
        return [a[o:o + c] for o, c in zip(self.offsets, self.counts)]


@dataclass
class LongRange:
    """Convenience: choose parameters and build a plan for a given system shape."""
    eps: float
    L: float
    n_max: int
    prec: str = "fp32"
    m: int = 0
    rc: float = 0.0
    tol_mode: str = "rel"
    q_l2: float = 0.0

    def __post_init__(self):
        self.params = choose_params(self.eps, self.L, rc=self.rc, m=self.m, n=self.n_max, q_l2=self.q_l2,
                                    tol_mode=self.tol_mode)
        self.plan = Plan(self.params, self.prec, self.n_max)

    def __call__(self, pos, q, **kw):
        return self.plan.compute(pos, q, **kw)
