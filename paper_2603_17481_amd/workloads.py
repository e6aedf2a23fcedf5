"""Parameters and seeded synthetic inputs for the coupled lattice step.

This module holds plain data only: the parameter record that both the GPU
binding and the oracle marshal into their own C structs, and the seeded
generators of initial conditions (droplet pairs, bubble swarms, slabs).  It
contains none of the method's update arithmetic.

Initial condition: phi = (1 + tanh(2 s / W)) / 2 with s the signed distance to
the nearest interface, positive in the liquid -- the equilibrium profile of
Sec. 2.2.4 (Eq. tanh_profile) with epsilon = W.  Node i sits at coordinate i;
distances use the periodic minimum image.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}


@dataclass
class Params:
    """Physical and numerical parameters of one lattice (lattice units).

    Names follow the paper: tau (Eq. nuomega), mobility M (= D of Eq. cace),
    width W (= epsilon = delta), sigma, density ratio rho_l/rho_g, a_rep
    (A_rep of Eq. Jrep_impl), body force g, and the detection parameters of
    Sec. 2.3.2 (w, q_th, eta, cos(theta_opp)) and Sec. 2.3.3 (h0, p, eps_n, eps_q).
    """

    dim: int = 2
    nx: int = 128
    ny: int = 128
    nz: int = 1
    precision: str = "fp64"
    tau: float = 1.0
    visc_ratio: float = 1.0
    mobility: float = 0.1
    width: float = 4.0
    sigma: float = 1e-3
    density_ratio: float = 1.0
    a_rep: float = 1e-3
    body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    nci_window: int = 3
    q_th: float = 0.125
    eta: float = 0.1
    cos_opp: float = -0.8
    h0: float = 1.0
    p_exp: float = 4.0
    eps_n: float = 1e-12
    eps_q: float = 1e-6
    tie_eps: float = 1e-6        # facing scores within tie_eps of the best count as tied
    rep_orient: int = 0          # 0: along n(x); +1: toward partner; -1: away from partner
    dispersed: int = -1          # 1: droplets {phi>1/2}; 0: bubbles {phi<1/2}; -1: minority phase
    cac_compress: int = 1        # 0 switches the counter-gradient flux off (diffusion test)
    cac_solver: int = 0          # phase field: 0 lattice Boltzmann (g), 1 finite-difference MUSCL-TVD
    hydro_q: int = 19            # 3D hydrodynamic lattice: D3Q19 or D3Q27 (2D is always D2Q9)
    hydro_store: int = 0         # 3D: 0 populations in place (AA), 1 post-collision moments
    diag_interval: int = 0       # periodic on-device diagnostics every K steps (0: never)
    pstar_ref: float = 0.0       # reference p* of the 16-bit population encoding

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * (self.nz if self.dim == 3 else 1)

    @property
    def shape(self) -> Tuple[int, ...]:
        """Array shape with x fastest: (ny, nx) in 2D, (nz, ny, nx) in 3D."""
        return (self.ny, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclass
class Sphere:
    center: Tuple[float, ...]
    radius: float
    velocity: Tuple[float, ...] = (0.0, 0.0, 0.0)


@dataclass
class InitialState:
    params: Params
    phi: np.ndarray                      # shape params.shape, float64
    u: np.ndarray                        # (dim,) + params.shape, float64
    spheres: List[Sphere] = field(default_factory=list)
    kind: str = ""


def _coords(p: Params):
    if p.dim == 2:
        y, x = np.meshgrid(np.arange(p.ny, dtype=np.float64), np.arange(p.nx, dtype=np.float64),
                           indexing="ij")
        return (x, y)
    z, y, x = np.meshgrid(np.arange(p.nz, dtype=np.float64), np.arange(p.ny, dtype=np.float64),
                          np.arange(p.nx, dtype=np.float64), indexing="ij")
    return (x, y, z)


def _min_image(d: np.ndarray, n: int) -> np.ndarray:
    return d - n * np.round(d / n)


def sphere_distance(p: Params, s: Sphere) -> np.ndarray:
    """Signed distance to the sphere surface (positive inside), periodic minimum image."""
    X = _coords(p)
    ns = (p.nx, p.ny, p.nz)
    r2 = np.zeros(p.shape)
    for a in range(p.dim):
        d = _min_image(X[a] - s.center[a], ns[a])
        r2 += d * d
    return s.radius - np.sqrt(r2)


def tanh_profile(s: np.ndarray, width: float) -> np.ndarray:
    return 0.5 * (1.0 + np.tanh(2.0 * s / width))


def spheres_state(p: Params, spheres: Sequence[Sphere], inside_liquid: bool = True,
                  kind: str = "") -> InitialState:
    """Union of spheres.  inside_liquid: droplets (phi=1 inside) else bubbles (phi=0 inside).

    The signed distance to the union is the largest per-sphere distance, so the
    profile follows the nearest surface (spheres are kept apart by the callers).
    """
    if spheres:
        dist = np.max(np.stack([sphere_distance(p, s) for s in spheres]), axis=0)
    else:
        dist = np.full(p.shape, -1e9)
    if not inside_liquid:
        dist = -dist
    phi = tanh_profile(dist, p.width)
    u = np.zeros((p.dim,) + p.shape)
    if inside_liquid:
        # u = sum_b phi_b U_b: each droplet carries its own velocity, the gas is at rest.
        for s in spheres:
            phib = tanh_profile(sphere_distance(p, s), p.width)
            for a in range(p.dim):
                u[a] += phib * s.velocity[a]
    return InitialState(p, phi, u, list(spheres), kind)


def droplet_pair(p: Params, radius: float, separation: float, speed: float,
                 offset: float = 0.0) -> InitialState:
    """Two equal droplets approaching along x with velocities +-speed.

    Centres sit at the box centre (N-1)/2 +- separation/2 along x and +-offset/2
    across it, so that the mirror planes of a symmetric set-up fall between nodes.
    """
    cx = (p.nx - 1) / 2.0
    cy = (p.ny - 1) / 2.0
    cz = (p.nz - 1) / 2.0 if p.dim == 3 else 0.0
    a = Sphere((cx - separation / 2.0, cy - offset / 2.0, cz), radius, (speed, 0.0, 0.0))
    b = Sphere((cx + separation / 2.0, cy + offset / 2.0, cz), radius, (-speed, 0.0, 0.0))
    return spheres_state(p, [a, b], True, "droplet_pair")


def static_droplet(p: Params, radius: float) -> InitialState:
    c = tuple((n - 1) / 2.0 for n in (p.nx, p.ny, p.nz))
    return spheres_state(p, [Sphere(c, radius)], True, "static_droplet")


def poisson_disk_spheres(p: Params, count: int, rmin: float, rmax: float, gap: float, seed: int,
                         max_tries: int = 200000) -> List[Sphere]:
    """Seeded dart throwing (numpy PCG64): radii uniform in [rmin, rmax], centres uniform,
    rejected when the periodic surface gap to an earlier sphere is below `gap`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.array([p.nx, p.ny, p.nz if p.dim == 3 else 1], dtype=np.float64)[: p.dim]
    centers = np.zeros((0, p.dim))
    radii = np.zeros(0)
    tries = 0
    while len(radii) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"placed only {len(radii)} of {count} spheres")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, 1.0, size=p.dim) * ns
        if len(radii):
            d = centers - c
            d -= ns * np.round(d / ns)
            dist = np.sqrt((d * d).sum(axis=1))
            if np.any(dist - radii - r < gap):
                continue
        centers = np.vstack([centers, c])
        radii = np.append(radii, r)
    out = []
    for c, r in zip(centers, radii):
        cc = tuple(float(v) for v in c) + (0.0,) * (3 - p.dim)
        out.append(Sphere(cc, float(r)))
    return out


def bubble_swarm(p: Params, count: int, rmin: float, rmax: float, gap: float, seed: int) -> InitialState:
    """Gas bubbles (phi = 0 inside) in liquid at rest."""
    sph = poisson_disk_spheres(p, count, rmin, rmax, gap, seed)
    st = _union_fast(p, sph, inside_liquid=False)
    st.kind = "bubble_swarm"
    return st


def _union_fast(p: Params, spheres: Sequence[Sphere], inside_liquid: bool) -> InitialState:
    """Same field as spheres_state, evaluated sphere by sphere on bounding boxes
    (needed for large boxes with many spheres).  Squared distances are formed
    per axis and summed in x, y, z order, as spheres_state does."""
    dist = np.full(p.shape, -1e30)
    ns = (p.nx, p.ny, p.nz)
    reach = p.width * 4.0
    for s in spheres:
        idx, contiguous = [], True
        for a in range(p.dim):
            lo_a = int(math.floor(s.center[a] - s.radius - reach))
            hi_a = int(math.ceil(s.center[a] + s.radius + reach))
            span = np.arange(lo_a, hi_a + 1)
            if len(span) >= ns[a]:
                span = np.arange(ns[a])
            ia = np.unique(np.mod(span, ns[a]))
            contiguous &= bool(ia[-1] - ia[0] + 1 == len(ia))
            idx.append(ia)
        d2 = [_min_image(idx[a].astype(np.float64) - s.center[a], ns[a]) ** 2 for a in range(p.dim)]
        if p.dim == 3:
            r2 = d2[0][None, None, :] + d2[1][None, :, None]
            r2 = r2 + d2[2][:, None, None]
        else:
            r2 = d2[0][None, :] + d2[1][:, None]
        d_s = s.radius - np.sqrt(r2)
        # arrays are indexed (z, y, x) / (y, x): reverse the axis order
        if contiguous:
            view = dist[tuple(slice(int(ia[0]), int(ia[-1]) + 1) for ia in idx[::-1])]
            np.maximum(view, d_s, out=view)
        else:
            ix = np.ix_(*idx[::-1])
            dist[ix] = np.maximum(dist[ix], d_s)
    dist = np.where(dist < -1e29, -1e3, dist)
    if not inside_liquid:
        dist = -dist
    phi = tanh_profile(dist, p.width)
    u = np.zeros((p.dim,) + p.shape)
    return InitialState(p, phi, u, list(spheres), "")


def slab(p: Params, thickness: float, axis: int = 0, center: Optional[float] = None,
         width: Optional[float] = None) -> InitialState:
    """Liquid slab (phi = 1 inside) of given thickness normal to `axis` (periodic)."""
    X = _coords(p)
    ns = (p.nx, p.ny, p.nz)
    c = (ns[axis] - 1) / 2.0 if center is None else center
    d = np.abs(_min_image(X[axis] - c, ns[axis]))
    s = thickness / 2.0 - d
    phi = tanh_profile(s, p.width if width is None else width)
    return InitialState(p, phi, np.zeros((p.dim,) + p.shape), [], "slab")


# ---------------------------------------------------------------------------
# The workloads the paper's experiments are restated as (lattice units).
# ---------------------------------------------------------------------------

def config_collision_2d(a_rep: float = 1e-3, precision: str = "fp64") -> InitialState:
    """2D head-on collision: 128x128 periodic, two droplets R=20, centres 50 apart,
    velocities +-0.05, density ratio 1, tau=1, W=4, sigma=1e-3, M=0.1."""
    p = Params(dim=2, nx=128, ny=128, nz=1, precision=precision, tau=1.0, mobility=0.1, width=4.0,
               sigma=1e-3, density_ratio=1.0, a_rep=a_rep)
    return droplet_pair(p, radius=20.0, separation=50.0, speed=0.05)


def config_collision_3d(offset_frac: float = 0.0, a_rep: float = 5e-3, precision: str = "fp32",
                        nx: int = 256, ny: int = 128, nz: int = 128, radius: float = 24.0,
                        separation: float = 64.0) -> InitialState:
    """3D head-on / off-axis collision: 256x128x128, droplets R=24 with centres 64 apart,
    velocities +-0.04, density ratio 10, viscosity ratio 1, W=5, sigma=5e-3."""
    p = Params(dim=3, nx=nx, ny=ny, nz=nz, precision=precision, tau=1.0, mobility=0.1, width=5.0,
               sigma=5e-3, density_ratio=10.0, a_rep=a_rep)
    return droplet_pair(p, radius=radius, separation=separation, speed=0.04,
                        offset=offset_frac * radius)


def config_swarm(n: int = 512, bubbles: int = 400, rmin: float = 8.0, rmax: float = 12.0,
                 gap: float = 3.0, seed: int = 3, precision: str = "fp32", a_rep: float = 5e-3,
                 gravity: float = 1e-6) -> InitialState:
    """Buoyant bubble swarm: n^3 periodic, seeded Poisson-disk bubbles, gravity along -z,
    density ratio 10, W=5, sigma=5e-3."""
    p = Params(dim=3, nx=n, ny=n, nz=n, precision=precision, tau=1.0, mobility=0.1, width=5.0,
               sigma=5e-3, density_ratio=10.0, a_rep=a_rep, body_force=(0.0, 0.0, -gravity),
               dispersed=0)
    return bubble_swarm(p, bubbles, rmin, rmax, gap, seed)
