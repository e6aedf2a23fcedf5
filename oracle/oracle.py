"""ctypes wrapper of the CPU FP64 oracle (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("tau", C.c_double), ("visc_ratio", C.c_double), ("mobility", C.c_double),
        ("width", C.c_double), ("sigma", C.c_double), ("density_ratio", C.c_double),
        ("a_rep", C.c_double), ("body_force", C.c_double * 3),
        ("nci_window", C.c_int),
        ("q_th", C.c_double), ("eta", C.c_double), ("cos_opp", C.c_double), ("h0", C.c_double),
        ("p_exp", C.c_double), ("eps_n", C.c_double), ("eps_q", C.c_double),
        ("tie_eps", C.c_double),
        ("rep_orient", C.c_int), ("dispersed", C.c_int), ("cac_compress", C.c_int),
        ("cac_solver", C.c_int), ("hydro_q", C.c_int), ("store_round", C.c_int),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("step", C.c_long), ("mass_phi", C.c_double), ("sum_pstar", C.c_double),
        ("momentum", C.c_double * 3), ("kinetic_energy", C.c_double), ("max_speed", C.c_double),
        ("n_droplets", C.c_long), ("nci_active", C.c_long), ("finite", C.c_int),
        ("film_frep_n", C.c_double), ("film_fcap_n", C.c_double), ("film_frep", C.c_double),
        ("max_frep", C.c_double),
    ]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from oracle import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    vp = C.c_void_p
    lib.oracle_create.restype = vp
    lib.oracle_create.argtypes = [C.POINTER(_Params)]
    lib.oracle_destroy.argtypes = [vp]
    lib.oracle_threads.restype = C.c_int
    lib.oracle_set_threads.restype = C.c_int
    lib.oracle_set_threads.argtypes = [C.c_int]
    for name in ("oracle_init_fields",):
        getattr(lib, name).argtypes = [vp, dp, dp, dp]
    lib.oracle_set_populations.argtypes = [vp, dp, dp]
    lib.oracle_set_rho_mean.argtypes = [vp, C.c_double]
    lib.oracle_set_phi.argtypes = [vp, dp]
    lib.oracle_get_populations.argtypes = [vp, dp, dp]
    lib.oracle_step.argtypes = [vp, C.c_int]
    lib.oracle_step_count.restype = C.c_long
    lib.oracle_step_count.argtypes = [vp]
    for name in ("oracle_get_phi", "oracle_get_rho", "oracle_get_pstar", "oracle_get_u",
                 "oracle_get_force"):
        getattr(lib, name).argtypes = [vp, dp]
    lib.oracle_get_nci.argtypes = [vp, ip, ip, dp]
    lib.oracle_get_gradients.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.oracle_diagnostics.argtypes = [vp, C.POINTER(_Diag)]
    lib.oracle_nci_from_qn.argtypes = [C.POINTER(_Params), dp, dp, ip, ip, dp]
    lib.oracle_feq.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
    lib.oracle_guo.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp]
    lib.oracle_regularize.argtypes = [C.c_int, C.c_int, dp, dp, dp]
    lib.oracle_film_thickness.restype = C.c_double
    lib.oracle_film_thickness.argtypes = [C.POINTER(_Params), C.c_double]
    lib.oracle_thickness_weight.restype = C.c_double
    lib.oracle_thickness_weight.argtypes = [C.POINTER(_Params), C.c_double]
    lib.oracle_count_components.restype = C.c_long
    lib.oracle_count_components.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_int]
    lib.oracle_component_sizes.restype = C.c_long
    lib.oracle_component_sizes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_int,
                                           C.POINTER(C.c_long), C.c_long]
    lib.oracle_lattice.argtypes = [C.c_int, ip, ip, dp, dp]
    _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_int))


def make_params(p, store_round: int = 0) -> _Params:
    s = _Params()
    s.dim, s.nx, s.ny = p.dim, p.nx, p.ny
    s.nz = p.nz if p.dim == 3 else 1
    s.tau, s.visc_ratio, s.mobility, s.width = p.tau, p.visc_ratio, p.mobility, p.width
    s.sigma, s.density_ratio, s.a_rep = p.sigma, p.density_ratio, p.a_rep
    for a in range(3):
        s.body_force[a] = float(p.body_force[a])
    s.nci_window = p.nci_window
    s.q_th, s.eta, s.cos_opp, s.h0 = p.q_th, p.eta, p.cos_opp, p.h0
    s.p_exp, s.eps_n, s.eps_q = p.p_exp, p.eps_n, p.eps_q
    s.tie_eps = p.tie_eps
    s.rep_orient, s.dispersed, s.cac_compress = p.rep_orient, p.dispersed, p.cac_compress
    s.cac_solver = p.cac_solver
    s.hydro_q = getattr(p, "hydro_q", 19) if p.dim == 3 else 9
    s.store_round = int(store_round)
    return s


def lattice(kind: int):
    """kind 0 = D2Q9, 1 = D3Q19, 2 = D3Q7, 3 = D3Q27 -> (c[q,3] int, w[q], cs2)."""
    lib = load()
    q = C.c_int()
    c = np.zeros(81, dtype=np.int32)
    w = np.zeros(27)
    cs2 = C.c_double()
    lib.oracle_lattice(kind, C.byref(q), _iptr(c), _dptr(w), C.byref(cs2))
    return c[: 3 * q.value].reshape(q.value, 3).copy(), w[: q.value].copy(), cs2.value


class Oracle:
    """One lattice on the CPU oracle.  Arrays follow Params.shape (x fastest)."""

    def __init__(self, params, store_round: int = 0):
        """store_round (test knob): 0 exact; 1/2/3 round the stored populations to
        float32 / half / bfloat16 after every step (sensitivity measurements)."""
        self.lib = load()
        self.params = params
        self._p = make_params(params, store_round)
        self.h = self.lib.oracle_create(C.byref(self._p))
        if not self.h:
            raise RuntimeError("oracle_create failed")
        self.N = params.n_cells
        self.dim = params.dim
        self.qf = 9 if params.dim == 2 else getattr(params, "hydro_q", 19)
        self.qg = 9 if params.dim == 2 else 7

    def close(self):
        if self.h:
            self.lib.oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, phi, u=None, pstar=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        pstar = None if pstar is None else np.ascontiguousarray(pstar, dtype=np.float64).reshape(-1)
        assert phi.size == self.N
        rc = self.lib.oracle_init_fields(self.h, _dptr(phi), _dptr(u), _dptr(pstar))
        if rc:
            raise RuntimeError("oracle_init_fields failed")

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        assert f.size == self.qf * self.N and g.size == self.qg * self.N
        self.lib.oracle_set_populations(self.h, _dptr(f), _dptr(g))

    def set_rho_mean(self, rho_mean: float):
        """Reference density of the buoyancy force for a sub-box of a larger box."""
        self.lib.oracle_set_rho_mean(self.h, float(rho_mean))

    def set_phi(self, phi):
        """Finite-difference phase field only: replace the stored phi."""
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        assert phi.size == self.N
        if self.lib.oracle_set_phi(self.h, _dptr(phi)):
            raise RuntimeError("oracle_set_phi needs cac_solver = 1")

    def get_populations(self):
        f = np.zeros(self.qf * self.N)
        g = np.zeros(self.qg * self.N)
        self.lib.oracle_get_populations(self.h, _dptr(f), _dptr(g))
        return f.reshape((self.qf,) + self.params.shape), g.reshape((self.qg,) + self.params.shape)

    def step(self, n: int = 1):
        if self.lib.oracle_step(self.h, int(n)):
            raise RuntimeError("oracle_step failed")

    @property
    def step_count(self) -> int:
        return int(self.lib.oracle_step_count(self.h))

    def _field(self, name, comps=1):
        out = np.zeros(comps * self.N)
        getattr(self.lib, name)(self.h, _dptr(out))
        shape = self.params.shape if comps == 1 else (comps,) + self.params.shape
        return out.reshape(shape)

    def phi(self):
        return self._field("oracle_get_phi")

    def rho(self):
        return self._field("oracle_get_rho")

    def pstar(self):
        return self._field("oracle_get_pstar")

    def u(self):
        return self._field("oracle_get_u", self.dim)

    def force(self):
        return self._field("oracle_get_force", self.dim)

    def gradients(self):
        """(grad phi, lap phi, n, q, mu_phi) of the current state."""
        d = self.dim
        g = np.zeros(d * self.N)
        lap = np.zeros(self.N)
        n = np.zeros(d * self.N)
        q = np.zeros(self.N)
        mu = np.zeros(self.N)
        self.lib.oracle_get_gradients(self.h, _dptr(g), _dptr(lap), _dptr(n), _dptr(q), _dptr(mu))
        sh = self.params.shape
        return (g.reshape((d,) + sh), lap.reshape(sh), n.reshape((d,) + sh), q.reshape(sh),
                mu.reshape(sh))

    def nci(self):
        chi = np.zeros(self.N, dtype=np.int32)
        part = np.zeros(3 * self.N, dtype=np.int32)
        J = np.zeros(self.dim * self.N)
        self.lib.oracle_get_nci(self.h, _iptr(chi), _iptr(part), _dptr(J))
        return (chi.reshape(self.params.shape), part.reshape((3,) + self.params.shape),
                J.reshape((self.dim,) + self.params.shape))

    def diagnostics(self) -> dict:
        d = _Diag()
        self.lib.oracle_diagnostics(self.h, C.byref(d))
        return {"step": d.step, "mass_phi": d.mass_phi, "sum_pstar": d.sum_pstar,
                "momentum": list(d.momentum)[: self.dim], "kinetic_energy": d.kinetic_energy,
                "max_speed": d.max_speed, "n_droplets": d.n_droplets, "nci_active": d.nci_active,
                "finite": bool(d.finite), "film_frep_n": d.film_frep_n, "film_fcap_n": d.film_fcap_n,
                "film_frep": d.film_frep, "max_frep": d.max_frep}


def nci_from_qn(params, q, n):
    """Detection + force of Sec. 2.3 on given q (shape) and n ((dim,)+shape) arrays."""
    lib = load()
    P = make_params(params)
    N = params.n_cells
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = np.ascontiguousarray(n, dtype=np.float64).reshape(-1)
    chi = np.zeros(N, dtype=np.int32)
    part = np.zeros(3 * N, dtype=np.int32)
    J = np.zeros(params.dim * N)
    lib.oracle_nci_from_qn(C.byref(P), _dptr(q), _dptr(n), _iptr(chi), _iptr(part), _dptr(J))
    return (chi.reshape(params.shape), part.reshape((3,) + params.shape),
            J.reshape((params.dim,) + params.shape))


def _hydro_q(dim, q):
    return 9 if dim == 2 else (q or 19)


def feq(dim, pstar, u, q=None):
    """Third-order equilibrium of one cell on D2Q9 (dim 2) or D3Q19 / D3Q27 (q)."""
    lib = load()
    q = _hydro_q(dim, q)
    out = np.zeros(q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    if lib.oracle_feq(dim, q, float(pstar), _dptr(uu), _dptr(out)):
        raise ValueError("unknown lattice")
    return out


def guo(dim, u, F, rho, q=None):
    lib = load()
    q = _hydro_q(dim, q)
    out = np.zeros(q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    FF = np.ascontiguousarray(F, dtype=np.float64)
    if lib.oracle_guo(dim, q, _dptr(uu), _dptr(FF), float(rho), _dptr(out)):
        raise ValueError("unknown lattice")
    return out


def regularize(dim, fneq, u, q=None):
    lib = load()
    q = _hydro_q(dim, q)
    out = np.zeros(q)
    a = np.ascontiguousarray(fneq, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    if lib.oracle_regularize(dim, q, _dptr(a), _dptr(uu), _dptr(out)):
        raise ValueError("unknown lattice")
    return out


def film_thickness(params, q):
    lib = load()
    P = make_params(params)
    return lib.oracle_film_thickness(C.byref(P), float(q))


def thickness_weight(params, h):
    lib = load()
    P = make_params(params)
    return lib.oracle_thickness_weight(C.byref(P), float(h))


def count_components(params, phi, dispersed):
    lib = load()
    a = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    nz = params.nz if params.dim == 3 else 1
    return int(lib.oracle_count_components(params.dim, params.nx, params.ny, nz, _dptr(a), dispersed))


def component_sizes(params, phi, dispersed):
    """Cell counts of the connected components (8- / 26-connected, periodic) of the
    dispersed set {phi > 1/2} (dispersed = 1) or {phi < 1/2} (0), largest first."""
    lib = load()
    a = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
    nz = params.nz if params.dim == 3 else 1
    cap = a.size
    out = np.zeros(cap, dtype=np.int64)
    n = int(lib.oracle_component_sizes(params.dim, params.nx, params.ny, nz, _dptr(a), dispersed,
                                       out.ctypes.data_as(C.POINTER(C.c_long)), cap))
    return np.sort(out[:n])[::-1]


def mean_curvature(params, n, dispersed):
    """Mean curvature kappa = div n_out (Eq. kappa_radius) of the interface of the
    dispersed phase, n_out its outward unit normal (n from Oracle.gradients(): grad phi
    over (|grad phi| + eps_n), so n_out = n for bubbles and -n for droplets), with the
    isotropic divergence (1/cs^2) sum_i w_i c_i . n_out(x + c_i) on the hydrodynamic
    lattice.  Written out literally with periodic shifts."""
    dim = params.dim
    kind = 0 if dim == 2 else (3 if getattr(params, "hydro_q", 19) == 27 else 1)
    c, w, cs2 = lattice(kind)
    sgn = 1.0 if dispersed == 0 else -1.0
    kappa = np.zeros(params.shape)
    axes = tuple(range(dim))[::-1]      # array axes of x, y, z (arrays are [z][y][x])
    for i in range(len(w)):
        shifted = 0.0
        for a in range(dim):
            if c[i][a] == 0:
                continue
            # n_out(x + c_i): roll by -c_i along every axis
            v = n[a]
            for b in range(dim):
                if c[i][b]:
                    v = np.roll(v, -int(c[i][b]), axis=axes[b])
            shifted = shifted + c[i][a] * v
        kappa += w[i] * shifted
    return sgn * kappa / cs2


def histogram_bins(values, lo, hi, nbins):
    """Bin index of each value: 0 below lo, nbins + 1 at or above hi, else
    1 + floor((v - lo) / (hi - lo) * nbins) (at most nbins)."""
    v = np.asarray(values, dtype=np.float64)
    b = 1 + np.minimum(nbins - 1, np.floor((v - lo) / (hi - lo) * nbins).astype(np.int64))
    b = np.where(v < lo, 0, b)
    return np.where(v >= hi, nbins + 1, b)
