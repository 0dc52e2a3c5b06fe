"""Seeded synthetic inputs for the patch-group MHM solver.

This module builds initial conserved states (rho, m_x, m_y, m_z, E) and lays
them out in the level storage the solver uses; it holds none of the solver's
arithmetic.  Both the HIP path and the CPU oracle take their inputs from here
and nothing else is shared between them.  The only physics evaluated here is
the ideal-gas total energy E = p/(gamma-1) + rho|v|^2/2 that turns each stated
initial pressure into the conserved energy the solver receives.

Level storage ("group-major"): the 16^3 interiors of all patch groups of one
level, float array [G, 5, 16, 16, 16], x fastest, with groups ordered
g = (gz*NGy + gy)*NGx + gx on an (NGx, NGy, NGz) lattice.  A patch group is the
2x2x2 set of sibling 8^3 patches that GAMER-2 sends to the GPU as one unit
(Sec. 3.1).

Random numbers: numpy Generator(PCG64(20171219 + config_id)).  Workloads:

  1  64^3 white-noise state, 64 groups, gamma = 5/3; and a Sod tube along x
     (n x 16 x 16 cells, outflow in x, periodic in y, z)
  2  256^3 shear layer (Kelvin-Helmholtz), 4096 groups, gamma = 1.4
  3  three uneven "AMR-shaped" levels of 512 / 1536 / 3072 groups with a
     Gaussian thermal-energy blast (Sedov-like), dx and dt halving per level
  4  128^3 smooth translating density wave, 512 groups, plus a noisy target
  5  384^3 supersonic-turbulence-like state, 13824 groups (log-normal density,
     k^-2 Gaussian random velocity field at rms Mach 3)

Every generator takes a size argument so that tests can run the same recipe at
sizes the oracle finishes in seconds.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

SEED_BASE = 20171219
N = 16  # cells per patch-group edge (2 x 8^3 patches per axis)

BC_PERIODIC = 0
BC_OUTFLOW = 1


def rng(config_id: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config_id))


@dataclass
class Level:
    """One level of patch groups plus the run parameters stated for it."""
    U: np.ndarray                       # [G, 5, 16, 16, 16] float64 (or float32)
    ng: Tuple[int, int, int]            # (NGx, NGy, NGz)
    dx: float
    gamma: float
    bc: Tuple[int, ...] = (0, 0, 0, 0, 0, 0)   # x-, x+, y-, y+, z-, z+
    meta: dict = field(default_factory=dict)

    @property
    def n_groups(self) -> int:
        return self.ng[0] * self.ng[1] * self.ng[2]

    @property
    def n_cells(self) -> int:
        return self.n_groups * N ** 3

    def astype(self, dtype) -> "Level":
        return Level(np.ascontiguousarray(self.U.astype(dtype)), self.ng, self.dx, self.gamma, self.bc,
                     dict(self.meta))


# ------------------------------------------------------------------ layout --

def grid_to_groups(a: np.ndarray) -> np.ndarray:
    """[5, Nz, Ny, Nx] -> group-major [G, 5, 16, 16, 16]."""
    f, Nz, Ny, Nx = a.shape
    ngz, ngy, ngx = Nz // N, Ny // N, Nx // N
    assert (ngz * N, ngy * N, ngx * N) == (Nz, Ny, Nx)
    b = a.reshape(f, ngz, N, ngy, N, ngx, N).transpose(1, 3, 5, 0, 2, 4, 6)
    return np.ascontiguousarray(b.reshape(ngz * ngy * ngx, f, N, N, N))


def groups_to_grid(u: np.ndarray, ng: Tuple[int, int, int]) -> np.ndarray:
    """group-major [G, 5, 16, 16, 16] -> [5, Nz, Ny, Nx]."""
    ngx, ngy, ngz = ng
    f = u.shape[1]
    b = u.reshape(ngz, ngy, ngx, f, N, N, N).transpose(3, 0, 4, 1, 5, 2, 6)
    return np.ascontiguousarray(b.reshape(f, ngz * N, ngy * N, ngx * N))


def conserved(rho, vx, vy, vz, p, gamma) -> np.ndarray:
    """Stack an initial (rho, v, p) state as conserved fields [5, ...]."""
    rho = np.asarray(rho, np.float64)
    shape = np.broadcast(rho, vx, vy, vz, p).shape
    rho, vx, vy, vz, p = (np.broadcast_to(np.asarray(a, np.float64), shape) for a in (rho, vx, vy, vz, p))
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, E])


def cell_centres(n: int, dx: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * dx


# --------------------------------------------------------------- workloads --

def white_noise(n: int = 64, config_id: int = 1, gamma: float = 5.0 / 3.0) -> Level:
    """Workload 1: rho ~ U(0.5, 2), v_i ~ N(0, 0.3), p ~ U(0.5, 2) per cell, periodic."""
    r = rng(config_id)
    shape = (n, n, n)
    rho = r.uniform(0.5, 2.0, shape)
    vx, vy, vz = (r.normal(0.0, 0.3, shape) for _ in range(3))
    p = r.uniform(0.5, 2.0, shape)
    U = grid_to_groups(conserved(rho, vx, vy, vz, p, gamma))
    return Level(U, (n // N,) * 3, 1.0 / n, gamma, meta={"name": "white-noise", "n": n})


def white_noise_device(ng: Tuple[int, int, int], dtype, device, config_id: int = 1, gamma: float = 5.0 / 3.0,
                       chunk: int = 4096):
    """Workload 1's white-noise recipe on an (NGx, NGy, NGz) lattice of any
    size, generated directly in device memory in level storage (a torch
    tensor [G, 5, 16, 16, 16] of `dtype`): for levels too large to build on
    the host.  Seeded with torch's device generator (SEED_BASE + config_id);
    the groups are drawn chunk by chunk, so the values depend on `chunk`."""
    import torch

    G = int(ng[0]) * int(ng[1]) * int(ng[2])
    U = torch.empty((G, 5, N, N, N), dtype=dtype, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_BASE + config_id)
    for g0 in range(0, G, chunk):
        n = min(chunk, G - g0)
        shape = (n, N, N, N)
        rho = torch.rand(shape, generator=gen, device=device, dtype=torch.float32) * 1.5 + 0.5
        v = [torch.randn(shape, generator=gen, device=device, dtype=torch.float32) * 0.3 for _ in range(3)]
        p = torch.rand(shape, generator=gen, device=device, dtype=torch.float32) * 1.5 + 0.5
        E = p / (gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
        blk = U[g0:g0 + n]
        blk[:, 0] = rho
        for i in range(3):
            blk[:, 1 + i] = rho * v[i]
        blk[:, 4] = E
    return U


def sod_tube(n: int = 128, gamma: float = 5.0 / 3.0, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
             axis: int = 0) -> Level:
    """Sod tube along `axis` (n cells, x in [0, 1], interface at 0.5), 16 cells across.

    Outflow at the two ends of the tube, periodic across it."""
    dx = 1.0 / n
    xc = cell_centres(n, dx)
    rho1 = np.where(xc < 0.5, left[0], right[0])
    u1 = np.where(xc < 0.5, left[1], right[1])
    p1 = np.where(xc < 0.5, left[2], right[2])
    dims = [N, N, N]
    dims[2 - axis] = n                                   # [Nz, Ny, Nx]
    shp = [1, 1, 1]
    shp[2 - axis] = n
    rho = np.broadcast_to(rho1.reshape(shp), dims)
    vel = [np.zeros(dims)] * 3
    vel[axis] = np.broadcast_to(u1.reshape(shp), dims)
    p = np.broadcast_to(p1.reshape(shp), dims)
    U = grid_to_groups(conserved(rho, vel[0], vel[1], vel[2], p, gamma))
    ng = [1, 1, 1]
    ng[axis] = n // N
    bc = [BC_PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = BC_OUTFLOW
    return Level(U, tuple(ng), dx, gamma, tuple(bc),
                 meta={"name": "sod", "n": n, "left": left, "right": right, "axis": axis})


def shear_layer(n: int = 256, config_id: int = 2, gamma: float = 1.4) -> Level:
    """Workload 2: rho = 2, v_x = +0.5 for |y - 1/2| >= 1/4; rho = 1, v_x = -0.5 inside;
    p = 2.5; v_y = 0.01 sin(4 pi x) + N(0, 1e-3).  Periodic, dx = 1/n."""
    r = rng(config_id)
    dx = 1.0 / n
    x = cell_centres(n, dx)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    inner = np.abs(Y - 0.5) < 0.25
    rho = np.where(inner, 1.0, 2.0)
    vx = np.where(inner, -0.5, 0.5)
    vy = 0.01 * np.sin(4.0 * np.pi * X) + r.normal(0.0, 1e-3, X.shape)
    U = grid_to_groups(conserved(rho, vx, vy, 0.0, 2.5, gamma))
    return Level(U, (n // N,) * 3, dx, gamma, meta={"name": "shear-layer", "n": n})


AMR_LEVEL_GROUPS = ((8, 8, 8), (8, 8, 24), (8, 16, 24))   # (NGx, NGy, NGz): 512, 1536, 3072


def sedov_levels(ng_levels=AMR_LEVEL_GROUPS, dx0: float = 1.0 / 128, gamma: float = 5.0 / 3.0,
                 e_blast: float = 1.0, p_bg: float = 1e-5) -> List[Level]:
    """Workload 3: one periodic brick of groups per level, dx_l = dx0 / 2^l.

    rho = 1, p = p_bg, plus thermal energy density exp(-r^2 / (2 sigma^2)) with
    sigma = 2 dx of the finest level, centred on the brick centre (a cell
    corner), rescaled on each level so that sum(E_th) dV = e_blast."""
    nl = len(ng_levels)
    sigma = 2.0 * dx0 / 2 ** (nl - 1)
    levels = []
    for l, ng in enumerate(ng_levels):
        dx = dx0 / 2 ** l
        nx, ny, nz = (k * N for k in ng)
        xs = [cell_centres(m, dx) - 0.5 * m * dx for m in (nz, ny, nx)]
        Z, Y, X = np.meshgrid(*xs, indexing="ij")
        g = np.exp(-(X * X + Y * Y + Z * Z) / (2.0 * sigma * sigma))
        eth = g * (e_blast / (g.sum() * dx ** 3))
        U = conserved(1.0, 0.0, 0.0, 0.0, p_bg, gamma)
        U = np.broadcast_to(U[:, None, None, None], (5, nz, ny, nx)).copy()
        U[4] += eth
        levels.append(Level(grid_to_groups(U), tuple(ng), dx, gamma,
                            meta={"name": "sedov", "level": l, "sigma": sigma}))
    return levels


# Workload 3 as a coupled hierarchy: level 0 is the 8^3-group domain; level l
# refines the level-(l-1) patches in a half-open box (patch indices of level
# l-1, x, y, z), mirror-symmetric about the domain centre: 16 x 12 x 8 = 1536
# level-1 groups and 24 x 16 x 8 = 3072 level-2 groups, each level nested in
# its parent with at least one parent patch of buffer.
AMR_NESTED_BOXES = (((0, 16), (2, 14), (4, 12)), ((4, 28), (8, 24), (12, 20)))


class AmrHierarchy:
    """Levels of a nested hierarchy: positions[l] [G_l, 3] (group lattice of
    level l: n0 * 2^l per axis), states[l] [G_l, 5, 16, 16, 16], dx0, bc."""

    def __init__(self, n0, positions, states, dx0, gamma, bc=(BC_PERIODIC,) * 6, meta=None):
        self.n0 = tuple(int(v) for v in n0)
        self.positions = [np.ascontiguousarray(p, np.int32) for p in positions]
        self.states = [np.ascontiguousarray(u) for u in states]
        self.dx0, self.gamma, self.bc = float(dx0), float(gamma), tuple(bc)
        self.meta = meta or {}

    @property
    def n_levels(self) -> int:
        return len(self.positions)

    def lattice(self, l: int) -> Tuple[int, int, int]:
        return tuple(v << l for v in self.n0)

    def dense_map(self, l: int) -> np.ndarray:
        """[n2, n1, n0] group index of level l at each lattice position, -1 if absent."""
        n = self.lattice(l)
        m = np.full((n[2], n[1], n[0]), -1, np.int32)
        p = self.positions[l]
        m[p[:, 2], p[:, 1], p[:, 0]] = np.arange(len(p), dtype=np.int32)
        return m

    def cells_per_coarse_step(self) -> int:
        return sum(len(p) * 4096 * 2 ** l for l, p in enumerate(self.positions))


def nested_positions(n0: int, boxes) -> List[np.ndarray]:
    """Level 0: all n0^3 groups (brick order, x fastest); level l: the children
    (one fine group each) of the level-(l-1) patches in boxes[l-1]."""
    out = [np.array([(x, y, z) for z in range(n0) for y in range(n0) for x in range(n0)], np.int32)]
    for bx, by, bz in boxes:
        out.append(np.array([(x, y, z) for z in range(*bz) for y in range(*by) for x in range(*bx)], np.int32))
    return out


def _level_cells(pos: np.ndarray, dx: float):
    """Cell-centre coordinates [G, 16, 16, 16] (x, y, z) of a level's groups."""
    i = (np.arange(N) + 0.5) * dx
    ox = pos[:, 0, None, None, None] * N * dx
    oy = pos[:, 1, None, None, None] * N * dx
    oz = pos[:, 2, None, None, None] * N * dx
    X = ox + i[None, None, None, :]
    Y = oy + i[None, None, :, None]
    Z = oz + i[None, :, None, None]
    return np.broadcast_arrays(X, Y, Z)


def restrict_states(h: "AmrHierarchy") -> None:
    """Coarse cells covered by a finer group take the mean of their children
    (finest level first), so that the initial hierarchy is consistent."""
    for l in range(h.n_levels - 1, 0, -1):
        cm = h.dense_map(l - 1)
        for g, (px, py, pz) in enumerate(h.positions[l]):
            f = h.states[l][g]
            c = f.reshape(5, 8, 2, 8, 2, 8, 2).mean(axis=(2, 4, 6))
            gc = cm[pz >> 1, py >> 1, px >> 1]
            h.states[l - 1][gc][:, (pz & 1) * 8:(pz & 1) * 8 + 8, (py & 1) * 8:(py & 1) * 8 + 8,
                                (px & 1) * 8:(px & 1) * 8 + 8] = c


def sedov_hierarchy(n0: int = 8, boxes=AMR_NESTED_BOXES, gamma: float = 5.0 / 3.0, e_blast: float = 1.0,
                    p_bg: float = 1e-5) -> AmrHierarchy:
    """Workload 3 on a coupled hierarchy: rho = 1, p = p_bg, thermal energy
    density exp(-r^2 / 2 sigma^2) with sigma = 2 cells of the finest level at
    the domain centre (a cell corner), normalized to e_blast on the finest
    level's cells; every level sampled at its cell centres, then coarse cells
    under finer groups replaced by their children's mean.  Unit domain:
    dx0 = 1 / (16 n0)."""
    dx0 = 1.0 / (N * n0)
    pos = nested_positions(n0, boxes)
    nl = len(pos)
    sigma = 2.0 * dx0 / 2 ** (nl - 1)
    states = []
    norm = None
    for l in range(nl - 1, -1, -1):
        dx = dx0 / 2 ** l
        X, Y, Z = _level_cells(pos[l], dx)
        r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
        g = np.exp(-r2 / (2.0 * sigma * sigma))
        if norm is None:
            norm = e_blast / (g.sum() * dx ** 3)
        U = np.empty((len(pos[l]), 5, N, N, N))
        U[:] = conserved(1.0, 0.0, 0.0, 0.0, p_bg, gamma)[None, :, None, None, None]
        U[:, 4] += g * norm
        states.insert(0, U)
    h = AmrHierarchy((n0,) * 3, pos, states, dx0, gamma, meta={"name": "sedov-amr", "sigma": sigma})
    restrict_states(h)
    return h


def smooth_wave(n: int = 128, config_id: int = 4, gamma: float = 5.0 / 3.0, amp: float = 0.01,
                v=(0.1, 0.05, 0.0), p0: float = 1.0, smooth_vp: float = 0.0) -> Tuple[Level, np.ndarray]:
    """Workload 4: rho = 1 + amp sin(2 pi (x+y+z)), uniform v and p (an exact
    translating solution).  Returns the level and a seeded target density
    rho_target = rho_0 + 0.01 N(0, 1) in group-major [G, 16, 16, 16].

    smooth_vp > 0 adds smooth variations of that amplitude to v and p, each
    varying along every axis (a variant for derivative checks: uniform fields
    put every velocity / pressure slope on the limiter's kink)."""
    r = rng(config_id)
    dx = 1.0 / n
    x = cell_centres(n, dx)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho = 1.0 + amp * np.sin(2.0 * np.pi * (X + Y + Z))
    tp = 2.0 * np.pi
    vx = v[0] + smooth_vp * np.sin(tp * (X + 2 * Y + Z) + 0.3)
    vy = v[1] + smooth_vp * np.cos(tp * (2 * X - Y + Z) + 0.7)
    vz = v[2] + smooth_vp * np.sin(tp * (X + Y - 2 * Z) + 1.1)
    pp = p0 + smooth_vp * np.cos(tp * (X + Y - Z) + 0.5)
    U = grid_to_groups(conserved(rho, vx, vy, vz, pp, gamma))
    target = rho + 0.01 * r.normal(0.0, 1.0, rho.shape)
    tgt = grid_to_groups(target[None])[:, 0]
    return Level(U, (n // N,) * 3, dx, gamma, meta={"name": "smooth-wave", "n": n, "v": v}), tgt


def smooth_wave_1d(n: int, gamma: float = 5.0 / 3.0, amp: float = 0.2, v=(1.0, 0.0, 0.0),
                   p0: float = 1.0, axis: int = 0) -> Level:
    """rho = 1 + amp sin(2 pi s) along one axis (n cells), 16 cells across; periodic."""
    dx = 1.0 / n
    s = cell_centres(n, dx)
    dims = [N, N, N]
    dims[2 - axis] = n
    shp = [1, 1, 1]
    shp[2 - axis] = n
    rho = np.broadcast_to((1.0 + amp * np.sin(2.0 * np.pi * s)).reshape(shp), dims)
    U = grid_to_groups(conserved(rho, v[0], v[1], v[2], p0, gamma))
    ng = [1, 1, 1]
    ng[axis] = n // N
    return Level(U, tuple(ng), dx, gamma, meta={"name": "smooth-wave-1d", "n": n, "amp": amp, "v": v})


def _grf(r: np.random.Generator, n: int, slope: float) -> np.ndarray:
    """Periodic Gaussian random field on n^3 with |f(k)|^2 ~ k^slope, zero mean, unit variance."""
    w = r.normal(0.0, 1.0, (n, n, n))
    fk = np.fft.rfftn(w)
    k1 = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (0.5 * slope)
    f = np.fft.irfftn(fk * amp, s=(n, n, n))
    f -= f.mean()
    return f / f.std()


def turbulence(n: int = 384, config_id: int = 5, gamma: float = 5.0 / 3.0, mach: float = 3.0) -> Level:
    """Workload 5: ln rho a GRF with sigma = 1 and mean -1/2; each velocity
    component an independent GRF with shell-integrated E(k) ~ k^-2 (so
    |v(k)|^2 ~ k^-4), scaled to rms |v| = mach * c_s with c_s = 1; p = rho/gamma."""
    r = rng(config_id)
    lnrho = _grf(r, n, -4.0) - 0.5
    rho = np.exp(lnrho)
    vel = [_grf(r, n, -4.0) for _ in range(3)]
    rms = np.sqrt(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    vel = [v * (mach / rms) for v in vel]
    U = grid_to_groups(conserved(rho, vel[0], vel[1], vel[2], rho / gamma, gamma))
    return Level(U, (n // N,) * 3, 1.0 / n, gamma, meta={"name": "turbulence", "n": n})
