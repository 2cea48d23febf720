"""Thin ctypes binding of libyeerom.so (argument marshalling only).

Every numerical step runs in the HIP library; this module converts numpy
arrays / torch tensors to the plain pointers and sizes of the C ABI declared
in ``include/yeerom.h``.  torch is used for device memory and streams only.
There is no fallback: if the library is not built, or no GPU is present,
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libyeerom.so")
_lib = None

YR_OK, YR_EINVAL, YR_ENOMEM, YR_EUNSTABLE, YR_ENOCONV, YR_EDEVICE, YR_ESTATE = 0, -1, -2, -3, -4, -5, -6
YR_F32, YR_F64 = 0, 1

_STATUS_NAMES = {YR_EINVAL: "EINVAL", YR_ENOMEM: "ENOMEM", YR_EUNSTABLE: "EUNSTABLE",
                 YR_ENOCONV: "ENOCONV", YR_EDEVICE: "EDEVICE", YR_ESTATE: "ESTATE"}


class YeeromError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.POINTER(C.c_double)), ("dy", C.POINTER(C.c_double)),
                ("dz", C.POINTER(C.c_double))]


class _Materials(C.Structure):
    _fields_ = [("eps_r", C.POINTER(C.c_double)), ("sigma_e", C.POINTER(C.c_double)),
                ("mu_r", C.POINTER(C.c_double)), ("sigma_m", C.POINTER(C.c_double)),
                ("n_pec", C.c_int64), ("pec", C.POINTER(C.c_int32))]


class _Ports(C.Structure):
    _fields_ = [("n", C.c_int32), ("offset", C.POINTER(C.c_int32)),
                ("sample", C.POINTER(C.c_int32)), ("weight", C.POINTER(C.c_double))]


def lib():
    """Load libyeerom.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built: run __graft_entry__.build() first")
    L = C.CDLL(_LIB_PATH)
    L.yr_last_error.restype = C.c_char_p
    vp = C.c_void_p
    L.yr_operator_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Materials), C.POINTER(vp)]
    L.yr_operator_destroy.argtypes = [vp]
    L.yr_operator_destroy.restype = None
    L.yr_operator_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.fdtd_step.argtypes = [vp, C.c_int, C.c_double, C.c_int64, vp, C.POINTER(_Ports), vp,
                            C.POINTER(_Ports), vp, vp]
    _bind_optional(L)
    _lib = L
    return L


class _MorOpts(C.Structure):
    _fields_ = [("M", C.c_double), ("L", C.c_int32), ("fmax", C.c_double),
                ("dt_ref", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("defl_tol", C.c_double), ("solve_dtype", C.c_int), ("matvec", C.c_int32),
                ("pair_only", C.c_int32)]


class _RomInfo(C.Structure):
    _fields_ = [("q1", C.c_int32), ("q2", C.c_int32), ("nsrc", C.c_int32), ("nprb", C.c_int32),
                ("deflated", C.c_int32), ("solve_iters", C.c_int64), ("matvecs", C.c_int64),
                ("relres_max", C.c_double), ("seconds_solve", C.c_double),
                ("seconds_orth", C.c_double), ("seconds_project", C.c_double),
                ("n_clamped", C.c_int32), ("step_dt", C.c_double), ("guard_margin", C.c_double)]


def _bind_optional(L):
    """Signatures of the entry points beyond the Yee operator."""
    vp = C.c_void_p
    sigs = {
        "mor_reduce": [vp, C.POINTER(_Ports), C.POINTER(_Ports), C.c_int32, C.POINTER(_MorOpts),
                       C.POINTER(vp)],
        "yr_rom_info": [vp, C.POINTER(_RomInfo)],
        "yr_rom_get": [vp, C.c_int32, C.POINTER(C.c_double)],
        "yr_rom_set": [vp, C.c_int32, C.POINTER(C.c_double)],
        "yr_rom_create": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)],
        "yr_rom_basis": [vp, vp, vp],
        "yr_rom_destroy": [vp],
        "yr_schur_apply": [vp, C.c_double, C.c_double, C.c_double, C.c_int, vp, vp, C.c_int32],
        "rom_perturb": [vp, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int32)],
        "rom_perturb_batch": [C.POINTER(vp), C.c_int32, C.c_double, C.c_double, C.c_int,
                              C.POINTER(C.c_int32)],
        "rom_step": [C.POINTER(vp), C.c_int32, C.c_double, C.c_int64, C.c_int, C.POINTER(vp),
                     C.POINTER(vp), C.POINTER(vp), vp],
        "rom_step_noalloc": [C.POINTER(vp), C.c_int32, C.c_double, C.c_int64, C.c_int,
                             C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp],
        "rom_lift": [vp, vp, C.c_int, C.c_int32, vp, vp, vp],
        "yr_operator_set_leapfrog": [vp, C.c_int32],
        "probe_dft": [C.c_int, vp, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_int32,
                      C.POINTER(C.c_double), C.c_int32, vp, vp],
        "fdtd_adjoint": [vp, C.c_int, C.c_double, C.c_int64, C.POINTER(_Ports), vp,
                         C.POINTER(_Ports), vp, C.c_int64, vp, vp, vp],
        "rom_adjoint": [vp, C.c_double, C.c_double, C.c_int64, vp, vp, C.POINTER(C.c_double),
                        C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                        C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "yr_rom_project_cells": [vp, vp, C.POINTER(C.c_double), C.c_int32,
                                 C.POINTER(C.c_double)],
        "yr_profile_enable": [C.c_int],
        "yr_profile_select": [C.c_char_p],
        "yr_profile_reset": [],
        "yr_profile_read": [C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    }
    for name, args in sigs.items():
        if hasattr(L, name):
            getattr(L, name).argtypes = args
    L.yr_rom_destroy.restype = None


def _check(status: int):
    if status != YR_OK:
        raise YeeromError(status, lib().yr_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def tensor_ptr(t) -> C.c_void_p:
    """Device pointer of a torch tensor (must be contiguous)."""
    if t is None:
        return C.c_void_p(0)
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check_tensor(t, name: str, dtype=None, numel=None, min_numel=None):
    """Reject what the C ABI cannot see: a dtype other than the call's, too few
    values for the sizes the call implies (the kernels would read or write
    past the end), or a strided view.  Host tensors are rejected by
    _on_device."""
    import torch
    if t is None:
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, the call needs {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} values, the call needs exactly {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} has {t.numel()} values, the call needs at least {min_numel}")
    return t


def _on_device(**tensors):
    """Every tensor handed to the library must be device memory (checked after
    the dtype and size checks of all arguments)."""
    for name, t in tensors.items():
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA (HIP device) tensor, got {t.device}")


def _torch_dtype(code: int):
    import torch
    return torch.float64 if code == YR_F64 else torch.float32


def stream_ptr(stream) -> C.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Ports:
    """CSR port list: each port a sequence of (c, i, j, k, weight) electric samples."""

    def __init__(self, ports: Sequence[Sequence[Tuple[int, int, int, int, float]]]):
        self.n = len(ports)
        off = [0]
        samples: List[int] = []
        weights: List[float] = []
        for port in ports:
            for (c, i, j, k, w) in port:
                samples += [int(c), int(i), int(j), int(k)]
                weights.append(float(w))
            off.append(len(weights))
        self._off = np.asarray(off, dtype=np.int32)
        self._smp = np.asarray(samples if samples else [0], dtype=np.int32)
        self._w = np.asarray(weights if weights else [0.0], dtype=np.float64)
        self.c = _Ports(self.n, _iptr(self._off), _iptr(self._smp), _dptr(self._w))

    def ref(self):
        return C.byref(self.c)


def _ports(p) -> Optional[Ports]:
    if p is None:
        return None
    return p if isinstance(p, Ports) else Ports(p)


class Operator:
    """Discretised structure (yr_operator): Sec. II-A, eq. (matrix)."""

    def __init__(self, dim: int, nx: int, ny: int, nz: int, dx, dy, dz=None, eps_r=None,
                 sigma_e=None, mu_r=None, sigma_m=None, pec=None):
        L = lib()
        self.dim, self.nx, self.ny, self.nz = int(dim), int(nx), int(ny), int(nz if dim == 3 else 1)
        keep = []

        def arr(a, n):
            if a is None:
                return None
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
            if a.size != n:
                raise ValueError(f"expected {n} values, got {a.size}")
            keep.append(a)
            return _dptr(a)

        ncell = self.nx * self.ny * self.nz
        g = _Grid(self.dim, self.nx, self.ny, self.nz, arr(dx, self.nx), arr(dy, self.ny),
                  arr(dz, self.nz) if self.dim == 3 else None)
        pec_arr = np.ascontiguousarray(np.asarray(pec if pec else [[0, 0, 0, 0]], dtype=np.int32))
        keep.append(pec_arr)
        m = _Materials(arr(eps_r, ncell), arr(sigma_e, ncell), arr(mu_r, ncell), arr(sigma_m, ncell),
                       len(pec) if pec else 0, _iptr(pec_arr))
        h = C.c_void_p()
        _check(L.yr_operator_create(C.byref(g), C.byref(m), C.byref(h)))
        self._h = h
        ln, ne, nh, dtm = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
        _check(L.yr_operator_info(h, C.byref(ln), C.byref(ne), C.byref(nh), C.byref(dtm)))
        self.len, self.n_e, self.n_h, self.dt_max = ln.value, ne.value, nh.value, dtm.value
        self.X, self.Y = self.nx + 1, self.ny + 1
        self.Z = self.nz + 1 if self.dim == 3 else 1
        self.ne_slots = 3 if self.dim == 3 else 1
        self.nh_slots = 3 if self.dim == 3 else 2

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.dim, wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz if wl.dim == 3 else None,
                   eps_r=wl.eps_r, sigma_e=wl.sigma_e, mu_r=wl.mu_r, sigma_m=wl.sigma_m,
                   pec=[list(p) for p in wl.pec] if wl.pec else None)

    @property
    def handle(self):
        return self._h

    @property
    def field_len(self) -> int:
        """Values in a full field buffer (E half then H half)."""
        return (self.ne_slots + self.nh_slots) * self.len

    def slot(self, c: int, i: int, j: int, k: int) -> int:
        """Offset of sample (c,i,j,k) in a field buffer (layout of yeerom.h)."""
        t = (k * self.Y + j) * self.X + i
        if self.dim == 2:
            s = {2: 0, 3: 1, 4: 2}[c]
        else:
            s = c
        return s * self.len + t

    def set_leapfrog(self, mode: str):
        """Leapfrog path of fdtd_step on a 3-D operator: "auto", "split" (two
        half-step kernels) or "fused" (one-pass steps)."""
        codes = {"auto": 0, "split": 1, "fused": 2}
        if mode not in codes:
            raise ValueError(f"mode must be one of {sorted(codes)}, got {mode!r}")
        _check(lib().yr_operator_set_leapfrog(self.handle, codes[mode]))

    def new_fields(self, dtype, device="cuda"):
        import torch
        return torch.zeros(self.field_len, dtype=dtype, device=device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yr_operator_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fdtd_adjoint(op: "Operator", dt: float, nsteps: int, src, u, probes, dJdy,
                 ckpt_every: int = 64, stream=None):
    """Gradients (dJ/d eps_r, dJ/d sigma_e) per cell, FP64 CUDA tensors shaped
    like the per-cell arrays ([nz, ny, nx] in 3-D, [ny, nx] in 2-D)."""
    import torch
    sp, pp = _ports(src), _ports(probes)
    if pp is None or pp.n < 1:
        raise ValueError("fdtd_adjoint needs at least one probe")
    code = _dtype_code(dJdy)
    _check_tensor(dJdy, "dJdy", min_numel=int(nsteps) * pp.n)
    if sp is not None and sp.n:
        _check_tensor(u, "u", dtype=_torch_dtype(code), min_numel=int(nsteps) * sp.n)
    _on_device(dJdy=dJdy, u=u if sp is not None and sp.n else None)
    shape = (op.nz, op.ny, op.nx) if op.dim == 3 else (op.ny, op.nx)
    ge = torch.zeros(shape, dtype=torch.float64, device="cuda")
    gs = torch.zeros(shape, dtype=torch.float64, device="cuda")
    _check(lib().fdtd_adjoint(op.handle, code, float(dt), int(nsteps),
                              sp.ref() if sp else None, tensor_ptr(u), pp.ref(),
                              tensor_ptr(dJdy), int(ckpt_every), tensor_ptr(ge), tensor_ptr(gs),
                              stream_ptr(stream)))
    return ge, gs


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return YR_F64
    if t.dtype == torch.float32:
        return YR_F32
    raise TypeError("fields must be float32 or float64")


def fdtd_step(op: Operator, dt: float, nsteps: int, fields, src=None, u=None, probes=None,
              y=None, stream=None):
    """Run ``nsteps`` leapfrog steps in place on ``fields`` (torch CUDA tensor).

    ``u``: [nsteps, n_src] tensor of the field dtype (u[n] drives E^{n+1});
    ``y``: [nsteps, n_probe] output tensor (y[n] = probe of E^{n+1}).
    """
    sp, pp = _ports(src), _ports(probes)
    code = _dtype_code(fields)
    _check_tensor(fields, "fields", numel=op.field_len)
    if sp is not None and sp.n:
        _check_tensor(u, "u", dtype=fields.dtype, min_numel=int(nsteps) * sp.n)
    if pp is not None and pp.n:
        _check_tensor(y, "y", dtype=fields.dtype, min_numel=int(nsteps) * pp.n)
    _on_device(fields=fields, u=u if sp is not None and sp.n else None,
               y=y if pp is not None and pp.n else None)
    _check(lib().fdtd_step(op.handle, code, float(dt), int(nsteps),
                           tensor_ptr(fields), sp.ref() if sp else None, tensor_ptr(u),
                           pp.ref() if pp else None, tensor_ptr(y), stream_ptr(stream)))


# ----------------------------------------------------------------------------- reduction

ROM_DE, ROM_DSE, ROM_DM, ROM_DSM, ROM_K, ROM_KP, ROM_B1, ROM_B2, ROM_L1, ROM_L2, ROM_SIGMA = range(11)


def _dtype_of(name) -> int:
    if name in ("f64", "float64", YR_F64):
        return YR_F64
    if name in ("f32", "float32", YR_F32):
        return YR_F32
    raise ValueError(f"unknown dtype {name!r}")


class Rom:
    """Reduced model (yr_rom): matrices of eq. (R_and_Freduced) + stepping data."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_matrices(cls, De, Dm, K, B1, L1, Dse=None, Dsm=None, B2=None, L2=None):
        De, Dm, K = (np.asarray(a, dtype=np.float64) for a in (De, Dm, K))
        q1, q2 = K.shape
        B1 = np.asarray(B1, dtype=np.float64).reshape(q1, -1)
        L1 = np.asarray(L1, dtype=np.float64).reshape(q1, -1)
        h = C.c_void_p()
        _check(lib().yr_rom_create(q1, q2, B1.shape[1], L1.shape[1], C.byref(h)))
        r = cls(h)
        r.set(ROM_DE, De)
        r.set(ROM_DM, Dm)
        r.set(ROM_K, K)
        r.set(ROM_B1, B1)
        r.set(ROM_L1, L1)
        if Dse is not None:
            r.set(ROM_DSE, Dse)
        if Dsm is not None:
            r.set(ROM_DSM, Dsm)
        if B2 is not None:
            r.set(ROM_B2, B2)
        if L2 is not None:
            r.set(ROM_L2, L2)
        return r

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _RomInfo()
        _check(lib().yr_rom_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in _RomInfo._fields_}

    def _shape(self, which):
        i = self.info()
        q1, q2, ns, npb = i["q1"], i["q2"], i["nsrc"], i["nprb"]
        return {ROM_DE: (q1, q1), ROM_DSE: (q1, q1), ROM_DM: (q2, q2), ROM_DSM: (q2, q2),
                ROM_K: (q1, q2), ROM_KP: (q1, q2), ROM_B1: (q1, ns), ROM_B2: (q2, ns),
                ROM_L1: (q1, npb), ROM_L2: (q2, npb), ROM_SIGMA: (min(q1, q2),)}[which]

    def get(self, which) -> np.ndarray:
        shp = self._shape(which)
        out = np.zeros(int(np.prod(shp)), dtype=np.float64)
        _check(lib().yr_rom_get(self._h, which, _dptr(out)))
        return out.reshape(shp[::-1]).T if len(shp) == 2 else out

    def set(self, which, a):
        shp = self._shape(which)
        a = np.asarray(a, dtype=np.float64).reshape(shp)
        buf = np.ascontiguousarray(a.T).ravel()  # column-major
        _check(lib().yr_rom_set(self._h, which, _dptr(buf)))

    def matrices(self) -> dict:
        names = {"De": ROM_DE, "Dse": ROM_DSE, "Dm": ROM_DM, "Dsm": ROM_DSM, "K": ROM_K,
                 "B1": ROM_B1, "B2": ROM_B2, "L1": ROM_L1, "L2": ROM_L2}
        return {k: self.get(v) for k, v in names.items()}

    def basis(self, op: "Operator"):
        """(V1, V2) as torch FP64 CUDA tensors [q, len*slots] (padded layout rows)."""
        import torch
        i = self.info()
        V1 = torch.zeros((i["q1"], op.ne_slots * op.len), dtype=torch.float64, device="cuda")
        V2 = torch.zeros((i["q2"], op.nh_slots * op.len), dtype=torch.float64, device="cuda")
        _check(lib().yr_rom_basis(self._h, tensor_ptr(V1), tensor_ptr(V2)))
        return V1, V2

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yr_rom_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mor_reduce(op: Operator, src, probes, q: int, dt_ref: float, fmax: float, M: float = 1.1,
               L: int = 2, tol: float = 1e-4, max_iter: int = 5000, defl_tol: float = 1e-10,
               precision="f32", matvec="auto", pair_only: bool = False) -> Rom:
    """Structure-preserving reduction (Sec. II-C, IV); see include/yeerom.h.

    ``matvec``: "auto" (the one-pass iteration where it applies), "two_sweep"
    or "one_pass" (the one-pass iteration wherever it exists).  ``pair_only``:
    expand at the conjugate pair M exp(+-j 2 pi fmax dt_ref) only (Sec. V-C)
    instead of eq. (distrib)."""
    sp, pp = _ports(src), _ports(probes)
    modes = {"auto": 0, "two_sweep": 1, "one_pass": 2}
    if matvec not in modes:
        raise ValueError(f"matvec must be 'auto', 'two_sweep' or 'one_pass', got {matvec!r}")
    o = _MorOpts(float(M), int(L), float(fmax), float(dt_ref), float(tol), int(max_iter),
                 float(defl_tol), _dtype_of(precision), modes[matvec], 1 if pair_only else 0)
    h = C.c_void_p()
    _check(lib().mor_reduce(op.handle, sp.ref(), pp.ref() if pp else None, int(q), C.byref(o),
                            C.byref(h)))
    return Rom(h)


def rom_perturb(roms, dt: float, gamma: float = 0.9999, dtype="f32"):
    """Sec. III-A singular-value clamp + stepping matrices for ``dt`` (batched).

    Returns the number of clamped singular values per model.
    """
    single = isinstance(roms, Rom)
    roms = [roms] if single else list(roms)
    arr = (C.c_void_p * len(roms))(*[r.handle for r in roms])
    ncl = (C.c_int32 * len(roms))()
    _check(lib().rom_perturb_batch(arr, len(roms), float(dt), float(gamma), _dtype_of(dtype), ncl))
    return ncl[0] if single else list(ncl)


def _step_args(roms, nsteps, us, ys, states, tdt):
    infos = [r.info() for r in roms]
    n = len(roms)
    us = list(us)
    if len(us) != n or len(ys) != n or (states is not None and len(states) != n):
        raise ValueError("one input, output (and state) per model")
    for m, i in enumerate(infos):
        if i["nsrc"] and us[m] is not None:
            _check_tensor(us[m], f"u[{m}]", dtype=tdt, min_numel=int(nsteps) * i["nsrc"])
        if i["nprb"]:
            _check_tensor(ys[m], f"y[{m}]", dtype=tdt, min_numel=int(nsteps) * i["nprb"])
        if states is not None and states[m] is not None:
            _check_tensor(states[m], f"state[{m}]", dtype=tdt, numel=i["q1"] + i["q2"])
    for m in range(n):
        _on_device(**{f"u[{m}]": us[m], f"y[{m}]": ys[m],
                      f"state[{m}]": states[m] if states is not None else None})
    arr = (C.c_void_p * n)(*[r.handle for r in roms])
    up = (C.c_void_p * n)(*[tensor_ptr(u).value if u is not None else None for u in us])
    yp = (C.c_void_p * n)(*[tensor_ptr(y).value for y in ys])
    sp_ = (C.c_void_p * n)(*[tensor_ptr(s).value for s in states]) if states is not None else None
    return n, arr, up, yp, sp_


def rom_step(roms, dt: float, nsteps: int, us, dtype="f32", states=None, ys=None, stream=None):
    """Reduced leapfrog of every model in one launch; returns the outputs y[m] [nsteps, nprb]."""
    import torch
    roms = list(roms)
    tdt = torch.float64 if _dtype_of(dtype) == YR_F64 else torch.float32
    if ys is None:
        ys = [torch.zeros((nsteps, max(r.info()["nprb"], 1)), dtype=tdt, device="cuda")
              for r in roms]
    n, arr, up, yp, sp_ = _step_args(roms, nsteps, us, ys, states, tdt)
    _check(lib().rom_step(arr, n, float(dt), int(nsteps), _dtype_of(dtype), up, yp, sp_,
                          stream_ptr(stream)))
    return ys


def rom_step_noalloc(roms, dt: float, nsteps: int, us, ys, dtype="f32", states=None,
                     stream=None):
    """rom_step through the entry point that allocates no device memory (for
    callers that cannot allocate): the caller provides every output buffer
    ys[m] [nsteps, nprb]; at most 4096 models per call; calls on one device
    must not overlap."""
    import torch
    roms = list(roms)
    tdt = torch.float64 if _dtype_of(dtype) == YR_F64 else torch.float32
    n, arr, up, yp, sp_ = _step_args(roms, nsteps, us, list(ys), states, tdt)
    _check(lib().rom_step_noalloc(arr, n, float(dt), int(nsteps), _dtype_of(dtype), up, yp,
                                  sp_, stream_ptr(stream)))
    return ys


def rom_lift(op: Operator, rom: "Rom", states, fields=None, stream=None):
    """Full fields x ~ V x~ from reduced states in rom_step's stepping
    coordinates (states: torch [nstates, q1+q2] or [q1+q2], FP32 or FP64).
    Returns torch [nstates, field_len] (or [field_len]) of the same dtype."""
    import torch
    single = states.dim() == 1
    st = states.reshape(1, -1) if single else states
    st = st.contiguous()
    i = rom.info()
    if st.shape[1] != i["q1"] + i["q2"]:
        raise ValueError(f"states have {st.shape[1]} entries, the model {i['q1'] + i['q2']}")
    dt_ = _dtype_code(st)
    _check_tensor(st, "states")
    if fields is None:
        fields = torch.zeros((st.shape[0], op.field_len), dtype=st.dtype, device=st.device)
    _check_tensor(fields, "fields", dtype=st.dtype, numel=st.shape[0] * op.field_len)
    _on_device(states=st, fields=fields)
    _check(lib().rom_lift(op.handle, rom.handle, dt_, int(st.shape[0]), tensor_ptr(st),
                          tensor_ptr(fields), stream_ptr(stream)))
    return fields[0] if single else fields


def probe_dft(y, dt: float, freqs, t0: float = 0.0, hann: bool = False, stream=None):
    """Spectra of probe records y [nsteps, nprb] (CUDA float32/float64), sample
    n at time t0 + n dt: Y[k, p] = dt sum_n w_n y[n, p] exp(-j 2 pi f_k t_n).
    Returns a CUDA complex128 tensor [len(freqs), nprb]."""
    import torch
    if y.dim() == 1:
        y = y.reshape(-1, 1)
    if y.dim() != 2:
        raise ValueError("y must be [nsteps, nprb]")
    code = _dtype_code(y)
    _check_tensor(y, "y")
    _on_device(y=y)
    f = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).ravel())
    out = torch.zeros((f.size, y.shape[1], 2), dtype=torch.float64, device=y.device)
    _check(lib().probe_dft(code, tensor_ptr(y), int(y.shape[0]), int(y.shape[1]), float(dt),
                           float(t0), int(f.size), _dptr(f), 1 if hann else 0, tensor_ptr(out),
                           stream_ptr(stream)))
    return torch.view_as_complex(out)


def schur_apply(op: Operator, dt: float, z: complex, x, dtype="f64"):
    """Test hook: y = S x for complex electric columns x (torch complex [ncol, ne_slots*len])."""
    import torch
    if not torch.is_complex(x) or x.dim() != 2 or x.shape[1] != op.ne_slots * op.len:
        raise ValueError("x must be a complex tensor [ncol, electric slots x len]")
    _check_tensor(x, "x")
    _on_device(x=x)
    y = torch.zeros_like(x)
    xr = torch.view_as_real(x).contiguous()
    yr_ = torch.view_as_real(y)
    _check(lib().yr_schur_apply(op.handle, float(dt), float(z.real), float(z.imag),
                                _dtype_of(dtype), tensor_ptr(xr), tensor_ptr(yr_), x.shape[0]))
    return y


def profile_enable(on: bool = True):
    _check(lib().yr_profile_enable(1 if on else 0))


def profile_select(names=None):
    """Time only the named kernels while profiling is on (None: all)."""
    arg = None if not names else ",".join(names).encode()
    _check(lib().yr_profile_select(arg))


def profile_reset():
    _check(lib().yr_profile_reset())


def profile_read(name: str):
    """(launches, total_ms) of a named kernel since the last reset."""
    n, ms = C.c_int64(), C.c_double()
    _check(lib().yr_profile_read(name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def rom_adjoint(rom: Rom, dt: float, nsteps: int, u, dJdy, dDe=None, through_clamp=True,
                gamma: float = 0.9999) -> dict:
    """Reduced adjoint (FP64): J, dJ/dtheta (clamp frozen / through the clamp),
    dJ/dDe~, dJ/dDse~, dJ/dK~'.  u, dJdy: FP64 CUDA tensors."""
    import torch
    i = rom.info()
    q1, q2 = i["q1"], i["q2"]
    if i["nsrc"]:
        _check_tensor(u, "u", dtype=torch.float64, min_numel=int(nsteps) * i["nsrc"])
    _check_tensor(dJdy, "dJdy", dtype=torch.float64, min_numel=int(nsteps) * i["nprb"])
    _on_device(u=u if i["nsrc"] else None, dJdy=dJdy)
    gDe = np.zeros(q1 * q1)
    gDse = np.zeros(q1 * q1)
    gK = np.zeros(q1 * q2)
    res = np.zeros(3)
    dd = None
    if dDe is not None:
        dd = np.ascontiguousarray(np.asarray(dDe, dtype=np.float64).T).ravel()
    _check(lib().rom_adjoint(rom.handle, float(dt), float(gamma), int(nsteps), tensor_ptr(u),
                             tensor_ptr(dJdy), _dptr(dd) if dd is not None else None,
                             1 if through_clamp else 0, _dptr(gDe), _dptr(gDse), _dptr(gK),
                             _dptr(res)))
    return {"J": res[0], "dJ_frozen": res[1], "dJ": res[2],
            "gDe": gDe.reshape(q1, q1).T, "gDse": gDse.reshape(q1, q1).T,
            "gK": gK.reshape(q2, q1).T}


def rom_project_cells(op: Operator, rom: Rom, cell_values, which: str = "eps") -> np.ndarray:
    """V1^T diag(W_e eps0 avg(cell_values)) V1 (which='eps') or with sigma (which='sigma')."""
    q1 = rom.info()["q1"]
    v = np.ascontiguousarray(np.asarray(cell_values, dtype=np.float64).ravel())
    out = np.zeros(q1 * q1)
    _check(lib().yr_rom_project_cells(op.handle, rom.handle, _dptr(v),
                                      0 if which == "eps" else 1, _dptr(out)))
    return out.reshape(q1, q1).T
