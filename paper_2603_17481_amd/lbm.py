"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice update runs in the HIP kernels of liblbm.so.  This
module only converts arrays and parameters; it raises if the library is
missing rather than computing anything itself.  PyTorch may supply the device
workspace and the stream (pass ``workspace=`` a CUDA tensor, ``stream=`` a
torch.cuda.Stream); otherwise the library allocates its own.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import List, Optional, Sequence

import numpy as np

from .workloads import PRECISIONS, Params

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK = 0
ERRORS = {-1: "LBM_E_INVALID", -2: "LBM_E_OOM", -3: "LBM_E_HIP", -4: "LBM_E_UNSUPPORTED",
          -5: "LBM_E_DIVERGED", -6: "LBM_E_STATE"}


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("precision", C.c_int),
        ("tau", C.c_double), ("visc_ratio", C.c_double), ("mobility", C.c_double),
        ("width", C.c_double), ("sigma", C.c_double), ("density_ratio", C.c_double),
        ("a_rep", C.c_double), ("body_force", C.c_double * 3),
        ("nci_window", C.c_int),
        ("q_th", C.c_double), ("eta", C.c_double), ("cos_opp", C.c_double),
        ("h0", C.c_double), ("p_exp", C.c_double),
        ("eps_n", C.c_double), ("eps_q", C.c_double), ("tie_eps", C.c_double),
        ("rep_orient", C.c_int), ("dispersed", C.c_int), ("cac_compress", C.c_int),
        ("diag_interval", C.c_int), ("pstar_ref", C.c_double), ("cac_solver", C.c_int),
        ("hydro_q", C.c_int), ("hydro_store", C.c_int),
    ]


class lbm_diag(C.Structure):
    _fields_ = [
        ("step", C.c_long), ("mass_phi", C.c_double), ("sum_pstar", C.c_double),
        ("momentum", C.c_double * 3), ("kinetic_energy", C.c_double), ("max_speed", C.c_double),
        ("n_droplets", C.c_long), ("nci_active", C.c_long), ("finite", C.c_int),
        ("film_cells", C.c_double), ("film_frep_n", C.c_double), ("film_fcap_n", C.c_double),
        ("film_frep", C.c_double), ("max_frep", C.c_double),
    ]


_lib = None


def load():
    """Load liblbm.so (built by paper_2603_17481_amd/build.py); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # One HIP runtime per process: torch's libraries ask for libamdhip64.so by its
    # file name, which a runtime loaded earlier under its versioned name does not
    # satisfy, so loading the library first would leave two runtimes that cannot
    # share the device.  With torch imported first, the library binds to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
    P = C.POINTER(lbm_params)
    lib.lbm_default_params.argtypes = [P]
    lib.lbm_default_params.restype = None
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = C.c_size_t
    lib.lbm_create.argtypes = [P, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_init_fields.argtypes = [vp, dp, dp, dp]
    lib.lbm_step.argtypes = [vp, C.c_int]
    lib.lbm_sync.argtypes = [vp]
    lib.lbm_step_count.argtypes = [vp]
    lib.lbm_step_count.restype = C.c_long
    for n in ("lbm_get_phi", "lbm_get_rho", "lbm_get_pstar", "lbm_get_u", "lbm_get_force"):
        getattr(lib, n).argtypes = [vp, dp]
    lib.lbm_get_nci.argtypes = [vp, ip, ip, dp]
    lib.lbm_diagnostics.argtypes = [vp, C.POINTER(lbm_diag)]
    lib.lbm_diag_history.argtypes = [vp, C.POINTER(lbm_diag), C.c_int]
    lib.lbm_lattice.argtypes = [C.c_int, C.c_int, ip]
    lib.lbm_get_populations.argtypes = [vp] + [C.c_int] * 6 + [dp, dp]
    lib.lbm_set_populations.argtypes = [vp, dp, dp]
    lib.lbm_state_bytes.argtypes = [vp]
    lib.lbm_state_bytes.restype = C.c_size_t
    lib.lbm_save_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbm_load_state.argtypes = [vp, vp, C.c_size_t]
    lib.lbm_batch_step.argtypes = [C.POINTER(vp), C.c_int, C.c_int]
    lib.lbm_batch_step_noalloc.argtypes = [C.POINTER(vp), C.c_int, C.c_int]
    lib.lbm_timing.argtypes = [vp, C.c_int]
    lib.lbm_kernel_times.argtypes = [vp, dp, C.POINTER(C.c_long)]
    lp = C.POINTER(C.c_long)
    lib.lbm_curvature_histogram.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int, lp]
    lib.lbm_component_volumes.argtypes = [vp, lp, C.c_long, lp]
    lib.lbm_force_wide_offsets.argtypes = [vp, C.c_int]
    lib.lbm_nci_select.argtypes = [vp, C.c_int]
    _lib = lib
    return lib


def header_functions() -> List[str]:
    """Names of the functions include/lbm.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def to_c_params(p: Params) -> lbm_params:
    s = lbm_params()
    load().lbm_default_params(C.byref(s))
    s.dim, s.nx, s.ny = p.dim, p.nx, p.ny
    s.nz = p.nz if p.dim == 3 else 1
    s.precision = PRECISIONS[p.precision]
    s.tau, s.visc_ratio, s.mobility, s.width = p.tau, p.visc_ratio, p.mobility, p.width
    s.sigma, s.density_ratio, s.a_rep = p.sigma, p.density_ratio, p.a_rep
    for a in range(3):
        s.body_force[a] = float(p.body_force[a])
    s.nci_window = p.nci_window
    s.q_th, s.eta, s.cos_opp, s.h0, s.p_exp = p.q_th, p.eta, p.cos_opp, p.h0, p.p_exp
    s.eps_n, s.eps_q, s.tie_eps = p.eps_n, p.eps_q, p.tie_eps
    s.rep_orient, s.dispersed, s.cac_compress = p.rep_orient, p.dispersed, p.cac_compress
    s.diag_interval = p.diag_interval
    s.pstar_ref = getattr(p, "pstar_ref", 0.0)
    s.cac_solver = getattr(p, "cac_solver", 0)
    hq = getattr(p, "hydro_q", 19)
    # 2D is always D2Q9: the 3D default passes as 0, anything else is refused by the library
    s.hydro_q = hq if p.dim == 3 or hq not in (9, 19) else 0
    s.hydro_store = getattr(p, "hydro_store", 0)
    return s


def lbm_workspace_bytes(p: Params) -> int:
    cp = to_c_params(p)
    return int(load().lbm_workspace_bytes(C.byref(cp)))


def lbm_lattice(dim: int, which: int) -> np.ndarray:
    lib = load()
    c = np.zeros(3 * 27, dtype=np.int32)
    q = lib.lbm_lattice(dim, which, c.ctypes.data_as(C.POINTER(C.c_int)))
    if q < 0:
        raise LBMError(q, "bad lattice")
    return c[: 3 * q].reshape(q, 3).copy()


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int))


def _diag_dict(d: lbm_diag, dim: int) -> dict:
    return {"step": d.step, "mass_phi": d.mass_phi, "sum_pstar": d.sum_pstar,
            "momentum": list(d.momentum)[:dim], "kinetic_energy": d.kinetic_energy,
            "max_speed": d.max_speed, "n_droplets": d.n_droplets, "nci_active": d.nci_active,
            "finite": bool(d.finite), "film_cells": d.film_cells, "film_frep_n": d.film_frep_n,
            "film_fcap_n": d.film_fcap_n, "film_frep": d.film_frep, "max_frep": d.max_frep}


class Lattice:
    """One lattice resident on the GPU (a context of the C ABI)."""

    def __init__(self, params: Params, workspace=None, stream=None):
        self.lib = load()
        self.params = params
        self._cp = to_c_params(params)
        self.N = params.n_cells
        self.dim = params.dim
        self.qf = 9 if params.dim == 2 else params.hydro_q
        self.qg = 9 if params.dim == 2 else 7
        self._workspace = workspace     # keep the tensor alive
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr = workspace.data_ptr()
            ws_bytes = workspace.numel() * workspace.element_size()
        st = None
        if stream is not None:
            st = getattr(stream, "cuda_stream", stream)
        h = C.c_void_p()
        rc = self.lib.lbm_create(C.byref(self._cp), ws_ptr, ws_bytes, st, C.byref(h))
        if rc != LBM_OK:
            raise LBMError(rc, self.lib.lbm_last_error(None).decode())
        self.h = h

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise LBMError(rc, self.lib.lbm_last_error(self.h).decode())
        return rc

    # -- state ------------------------------------------------------------
    def init_fields(self, phi, u=None, pstar=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        if phi.size != self.N:
            raise ValueError("phi has the wrong size")
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        ps = None if pstar is None else np.ascontiguousarray(pstar, dtype=np.float64).reshape(-1)
        if uu is not None and uu.size != self.dim * self.N:
            raise ValueError("u has the wrong size")
        self._check(self.lib.lbm_init_fields(self.h, _dp(phi), _dp(uu), _dp(ps)))

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.lbm_sync(self.h))

    @property
    def step_count(self) -> int:
        return int(self.lib.lbm_step_count(self.h))

    def _field(self, name: str, comps: int = 1):
        out = np.zeros(comps * self.N)
        self._check(getattr(self.lib, name)(self.h, _dp(out)))
        sh = self.params.shape
        return out.reshape(sh if comps == 1 else (comps,) + sh)

    def phi(self):
        return self._field("lbm_get_phi")

    def rho(self):
        return self._field("lbm_get_rho")

    def pstar(self):
        return self._field("lbm_get_pstar")

    def u(self):
        return self._field("lbm_get_u", self.dim)

    def force(self):
        return self._field("lbm_get_force", self.dim)

    def nci(self):
        chi = np.zeros(self.N, dtype=np.int32)
        part = np.zeros(3 * self.N, dtype=np.int32)
        J = np.zeros(self.dim * self.N)
        self._check(self.lib.lbm_get_nci(self.h, _ip(chi), _ip(part), _dp(J)))
        sh = self.params.shape
        return chi.reshape(sh), part.reshape((3,) + sh), J.reshape((self.dim,) + sh)

    def diagnostics(self) -> dict:
        d = lbm_diag()
        self._check(self.lib.lbm_diagnostics(self.h, C.byref(d)))
        return _diag_dict(d, self.dim)

    def diag_history(self, max_entries: int = 64) -> List[dict]:
        arr = (lbm_diag * max_entries)()
        n = self._check(self.lib.lbm_diag_history(self.h, arr, max_entries))
        return [_diag_dict(arr[i], self.dim) for i in range(n)]

    def get_populations(self, x0=0, y0=0, z0=0, bx=None, by=None, bz=None):
        p = self.params
        bx = p.nx if bx is None else bx
        by = p.ny if by is None else by
        bz = (p.nz if p.dim == 3 else 1) if bz is None else bz
        B = bx * by * bz
        f = np.zeros(self.qf * B)
        g = np.zeros(self.qg * B)
        self._check(self.lib.lbm_get_populations(self.h, x0, y0, z0, bx, by, bz, _dp(f), _dp(g)))
        sh = (by, bx) if p.dim == 2 else (bz, by, bx)
        return f.reshape((self.qf,) + sh), g.reshape((self.qg,) + sh)

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        if f.size != self.qf * self.N or g.size != self.qg * self.N:
            raise ValueError("population arrays have the wrong size")
        self._check(self.lib.lbm_set_populations(self.h, _dp(f), _dp(g)))

    def timing(self, enable: bool = True):
        self._check(self.lib.lbm_timing(self.h, 1 if enable else 0))

    def curvature_histogram(self, q_band: float, kmin: float, kmax: float, nbins: int) -> np.ndarray:
        """Counts of the interfacial mean curvature: [below kmin, nbins bins, at or above kmax]."""
        out = np.zeros(nbins + 2, dtype=np.int64)
        self._check(self.lib.lbm_curvature_histogram(self.h, float(q_band), float(kmin), float(kmax), int(nbins),
                                                     out.ctypes.data_as(C.POINTER(C.c_long))))
        return out

    def component_volumes(self, max_count: int = 1 << 20) -> np.ndarray:
        """Cell counts of the dispersed components, largest first."""
        out = np.zeros(max_count, dtype=np.int64)
        n = C.c_long()
        self._check(self.lib.lbm_component_volumes(self.h, out.ctypes.data_as(C.POINTER(C.c_long)), int(max_count),
                                                   C.byref(n)))
        if n.value > max_count:
            raise LBMError(-1, f"{n.value} components, more than max_count = {max_count}")
        return out[: n.value].copy()

    def nci_select(self, mode: int):
        """Near-contact tile selection: -1 by lattice size (default), 0 never, 1 always."""
        self._check(self.lib.lbm_nci_select(self.h, int(mode)))

    def force_wide_offsets(self, on: bool = True):
        """Testing hook: run the collide kernels with 64-bit element offsets."""
        self._check(self.lib.lbm_force_wide_offsets(self.h, 1 if on else 0))

    def kernel_times(self):
        """{kernel: (total_ms, launches)} since the last call (synchronises)."""
        ms = np.zeros(5)
        cnt = (C.c_long * 5)()
        self._check(self.lib.lbm_kernel_times(self.h, _dp(ms), cnt))
        names = ("phi", "nci", "collide", "diag", "muscl")
        return {names[k]: (float(ms[k]), int(cnt[k])) for k in range(5)}

    def save_state(self) -> bytes:
        n = int(self.lib.lbm_state_bytes(self.h))
        buf = C.create_string_buffer(n)
        self._check(self.lib.lbm_save_state(self.h, buf, n))
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(self.lib.lbm_load_state(self.h, buf, len(data)))


def lbm_batch_step(lattices: Sequence[Lattice], n: int):
    """Advance several resident lattices together (multi-domain launches)."""
    if not lattices:
        return
    lib = lattices[0].lib
    arr = (C.c_void_p * len(lattices))(*[lt.h for lt in lattices])
    rc = lib.lbm_batch_step(arr, len(lattices), int(n))
    if rc < 0:
        raise LBMError(rc, lib.lbm_last_error(lattices[0].h).decode())


def lbm_batch_step_noalloc(lattices: Sequence[Lattice], n: int):
    """lbm_batch_step without any device allocation (static job table, no graph;
    synchronous); at most 64 lattices."""
    if not lattices:
        return
    lib = lattices[0].lib
    arr = (C.c_void_p * len(lattices))(*[lt.h for lt in lattices])
    rc = lib.lbm_batch_step_noalloc(arr, len(lattices), int(n))
    if rc < 0:
        raise LBMError(rc, lib.lbm_last_error(lattices[0].h).decode())
