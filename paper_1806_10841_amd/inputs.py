"""Seeded synthetic inputs for the adaptive-resolution (AdResS) hot path.

This module only *places* particles and draws random numbers: lattices,
random rigid orientations, Maxwell-Boltzmann velocities and lattice polymer
chains.  It contains none of the method's arithmetic (no resolution weights,
no forces, no lists, no integration), so that the FP64 oracle and the HIP
library can both be fed from it without sharing any computation.

Layout of every state array: float64, structure-of-arrays, shape (3, N_s),
row 0/1/2 = x/y/z.  Molecule ``a`` owns the ``s`` consecutive sites
``a*s .. a*s+s-1`` (tetrahedra: s = 4; beads and CG sites: s = 1).

Workloads (all lengths in units of the atom diameter sigma):

* ``c1``  512 tetrahedra, 8^3 lattice, L = 17.1, x-slab AT half-width 4, hybrid 3, FP64.
* ``c2``  64,000 tetrahedra (256,000 atoms), 40^3 lattice, molecular density 0.1
          (L = 86.177), x-slab AT half-width 10, hybrid 5, FP32 pair arithmetic.
* ``c3``  Kremer-Grest-type melt: 1000 chains x 200 beads, bead density 0.85,
          FENE (k=30, R0=1.5) + WCA on every pair, 1-site "molecules", all atomistic.
* ``c4``  256,000 coarse-grained sites (C2 density, box tiled 2x2x1), all CG,
          CG force from a learned MLP or a tabulated cubic spline, cutoff 3.0.
* ``c5``  1,000,000 tetrahedra (4M atoms), sphere AT radius 12 + hybrid shell 5.

``tiny``- and ``small``-prefixed workloads are scaled-down versions used by the tests;
``small_dumbbell`` and ``small_triangle`` hold 2- and 3-site molecules (unit bonds).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict, replace

import numpy as np

# Regions of the resolution function (which molecules are atomistic).
REGION_ALL_AT = 0   # w == 1 everywhere (plain atomistic MD)
REGION_SLAB_X = 1   # AT slab centred at box centre, normal along x
REGION_SPHERE = 2   # AT sphere centred at the box centre
REGION_ALL_CG = 3   # w == 0 everywhere (plain coarse-grained MD)
REGION_SPHERES = 4  # AT region = union of spheres around the centres of anchor molecules

CG_WCA = 0      # analytic WCA between centres of mass
CG_TABLE = 1    # cubic-spline table of the CG force
CG_MLP = 2      # learned MLP, BF16 matrix cores
CG_MLP_FP8 = 3  # the same network with layer 2 on FP8 E4M3 matrix cores

SCHEME_FORCE = 0        # force interpolation, Eq. (1)
SCHEME_HAMILTONIAN = 1  # potential energy interpolation, Eq. (2) (H-AdResS)
BOND_NONE = 0
BOND_HARMONIC = 1   # harmonic bonds between every pair of sites of a molecule
BOND_FENE = 2       # FENE bonds between consecutive beads of a chain

WCA_RC = 2.0 ** (1.0 / 6.0)


@dataclass
class Workload:
    """Physical parameters of one synthetic workload (plain data, no arithmetic)."""
    name: str
    n_mol: int
    sites_per_mol: int
    box: tuple
    site_mass: tuple
    region: int
    center: tuple
    d_at: float
    d_hy: float
    eps_at: float = 1.0
    sig_at: float = 1.0
    rc_at: float = WCA_RC
    eps_cg: float = 1.0
    sig_cg: float = 2.31
    rc_cg: float = WCA_RC * 2.31
    cg_kind: int = CG_WCA
    bond_kind: int = BOND_HARMONIC
    k_bond: float = 400.0
    r0_bond: float = 1.0
    chain_len: int = 0
    r_skin: float = 0.3
    rho_max: float = 0.8
    pair_precision: int = 64
    dt: float = 0.005
    n_steps: int = 100
    gamma: float = 0.0
    kT: float = 1.0
    seed: int = 1000
    scheme: int = SCHEME_FORCE

    def as_dict(self):
        return asdict(self)

    def with_(self, **kw):
        return replace(self, **kw)


def _tetra_body():
    """Vertices of a regular tetrahedron with unit edge, centred at the origin."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    return v / (2.0 * math.sqrt(2.0))


def random_rotations(n, rng):
    """Uniform random rotation matrices (Shoemake's quaternion method), shape (n,3,3)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    q0 = a * np.sin(2 * np.pi * u2)
    q1 = a * np.cos(2 * np.pi * u2)
    q2 = b * np.sin(2 * np.pi * u3)
    q3 = b * np.cos(2 * np.pi * u3)
    # quaternion (w=q3, x=q0, y=q1, z=q2) -> matrix
    w, x, y, z = q3, q0, q1, q2
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def wrap_into_box(x, box):
    """Fold coordinates into [0, L) per dimension (x: (3, N))."""
    x = np.array(x, dtype=np.float64, copy=True)
    for d in range(3):
        L = box[d]
        x[d] = np.mod(x[d], L)
        x[d][x[d] >= L] -= L   # np.mod can round up to L for tiny negatives
    return x


def lattice_points(dims, box, rng=None, jitter=0.0):
    """Simple-cubic lattice sites at cell centres, optionally jittered: (3, prod(dims))."""
    nx, ny, nz = dims
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([(ix.ravel() + 0.5) * (box[0] / nx),
                    (iy.ravel() + 0.5) * (box[1] / ny),
                    (iz.ravel() + 0.5) * (box[2] / nz)])
    if jitter > 0.0:
        pts = pts + rng.uniform(-jitter, jitter, size=pts.shape)
    return pts


def tetra_positions(com, rng):
    """Sites of randomly oriented unit-edge tetrahedra around the given centres.

    com: (3, n_mol).  Returns unwrapped (3, 4*n_mol) site positions."""
    n = com.shape[1]
    rot = random_rotations(n, rng)
    body = _tetra_body()                      # (4, 3)
    offs = np.einsum("nij,kj->nki", rot, body)  # (n, 4, 3)
    pos = com.T[:, None, :] + offs            # (n, 4, 3)
    return pos.reshape(n * 4, 3).T.copy()


def _small_body(spm):
    """Unit-edge rigid bodies centred at the origin: a dumbbell (2 sites) or an equilateral
    triangle (3 sites), shape (spm, 3)."""
    if spm == 2:
        return np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    if spm == 3:
        R = 1.0 / math.sqrt(3.0)   # circumradius of the unit triangle
        return np.array([[0.0, R, 0.0], [-0.5, -0.5 * R, 0.0], [0.5, -0.5 * R, 0.0]])
    raise ValueError(spm)


def body_positions(com, spm, rng):
    """Sites of randomly oriented dumbbells (spm 2) or triangles (spm 3) around the given
    centres, com: (3, n_mol).  Returns unwrapped (3, spm*n_mol) site positions."""
    n = com.shape[1]
    rot = random_rotations(n, rng)
    offs = np.einsum("nij,kj->nki", rot, _small_body(spm))
    return (com.T[:, None, :] + offs).reshape(n * spm, 3).T.copy()


def maxwell_velocities(n_sites, masses, kT, rng):
    """Maxwell-Boltzmann velocities at temperature kT with the total momentum removed."""
    m = np.asarray(masses, dtype=np.float64)
    v = rng.normal(size=(3, n_sites)) * np.sqrt(kT / m)[None, :]
    p = (v * m[None, :]).sum(axis=1) / m.sum()
    return v - p[:, None]


def serpentine_path(n):
    """A Hamiltonian path with unit steps through an n^3 simple-cubic lattice."""
    out = []
    row = 0
    for z in range(n):
        ys = range(n) if z % 2 == 0 else range(n - 1, -1, -1)
        for y in ys:
            xs = range(n) if row % 2 == 0 else range(n - 1, -1, -1)
            for x in xs:
                out.append((x, y, z))
            row += 1
    return np.array(out, dtype=np.int64)


def workload(name: str) -> Workload:
    """Named workloads.  Lengths in sigma, energies in epsilon, masses in atom masses."""
    tetra_mass = (1.0, 1.0, 1.0, 1.0)
    if name == "c1":
        L = 17.1
        return Workload("c1", 512, 4, (L, L, L), tetra_mass, REGION_SLAB_X, (L / 2, L / 2, L / 2),
                        4.0, 3.0, pair_precision=64, n_steps=100, seed=1001)
    if name == "c2":
        L = (64000 / 0.1) ** (1.0 / 3.0)
        return Workload("c2", 64000, 4, (L, L, L), tetra_mass, REGION_SLAB_X, (L / 2, L / 2, L / 2),
                        10.0, 5.0, pair_precision=32, n_steps=1000, seed=1002)
    if name == "c3":
        L = (200000 / 0.85) ** (1.0 / 3.0)
        return Workload("c3", 200000, 1, (L, L, L), (1.0,), REGION_ALL_AT, (L / 2, L / 2, L / 2),
                        0.0, 0.0, bond_kind=BOND_FENE, k_bond=30.0, r0_bond=1.5, chain_len=200,
                        rho_max=0.0, pair_precision=32, dt=0.01, n_steps=1000,
                        gamma=0.5, kT=1.0, seed=1003, r_skin=0.5)   # (no skin stated: a tuning choice)
    if name == "c4":
        L = (64000 / 0.1) ** (1.0 / 3.0)
        return Workload("c4", 256000, 1, (2 * L, 2 * L, L), (4.0,), REGION_ALL_CG,
                        (L, L, L / 2), 0.0, 0.0, rc_cg=3.0, cg_kind=CG_MLP,
                        bond_kind=BOND_NONE, rho_max=0.0, pair_precision=32,
                        n_steps=1000, seed=1004)
    if name == "c5":
        L = (1000000 / 0.1) ** (1.0 / 3.0)
        return Workload("c5", 1000000, 4, (L, L, L), tetra_mass, REGION_SPHERE, (L / 2, L / 2, L / 2),
                        12.0, 5.0, cg_kind=CG_TABLE, pair_precision=32, n_steps=500, seed=1005,
                        r_skin=0.5)   # (no skin stated: a tuning choice)
    # scaled-down variants for CPU tests (same physics, fewer molecules)
    if name == "tiny_slab":      # 4^3 tetrahedra, every resolution present
        L = 4 * 2.15
        return Workload("tiny_slab", 64, 4, (L, L, L), tetra_mass, REGION_SLAB_X, (L / 2, L / 2, L / 2),
                        1.05, 1.5, pair_precision=64, n_steps=20, seed=7)
    if name == "small_slab":     # 10^3 tetrahedra at C2 density
        L = (1000 / 0.1) ** (1.0 / 3.0)
        return Workload("small_slab", 1000, 4, (L, L, L), tetra_mass, REGION_SLAB_X,
                        (L / 2, L / 2, L / 2), 3.0, 2.0, pair_precision=64, n_steps=50, seed=8)
    if name == "small_sphere":
        L = (1728 / 0.1) ** (1.0 / 3.0)
        return Workload("small_sphere", 1728, 4, (L, L, L), tetra_mass, REGION_SPHERE,
                        (L / 2, L / 2, L / 2), 4.0, 3.0, pair_precision=64, n_steps=20, seed=9)
    if name in ("small_dumbbell", "small_triangle"):   # 2- and 3-site molecules, 10^3
        # denser than C2 with a narrower CG site (sigma 1.75), so that atom pairs of
        # neighbouring molecules are inside the WCA cutoff and lattice neighbours interact
        spm = 2 if name == "small_dumbbell" else 3
        L = (1000 / 0.15) ** (1.0 / 3.0)
        return Workload(name, 1000, spm, (L, L, L), (1.0,) * spm, REGION_SLAB_X, (L / 2, L / 2, L / 2),
                        3.0, 2.0, sig_cg=1.75, rc_cg=WCA_RC * 1.75, pair_precision=64, n_steps=50,
                        seed=12 + spm)
    if name == "small_kg":
        L = (4000 / 0.85) ** (1.0 / 3.0)
        return Workload("small_kg", 4000, 1, (L, L, L), (1.0,), REGION_ALL_AT, (L / 2, L / 2, L / 2),
                        0.0, 0.0, bond_kind=BOND_FENE, k_bond=30.0, r0_bond=1.5, chain_len=50,
                        rho_max=0.0, pair_precision=64, dt=0.01, n_steps=50, seed=10)
    if name == "small_cg":
        L = (2197 / 0.1) ** (1.0 / 3.0)
        return Workload("small_cg", 2197, 1, (L, L, L), (4.0,), REGION_ALL_CG, (L / 2, L / 2, L / 2),
                        0.0, 0.0, rc_cg=3.0, cg_kind=CG_TABLE, bond_kind=BOND_NONE, rho_max=0.0,
                        pair_precision=64, n_steps=50, seed=11)
    raise KeyError(name)


def _lattice_dims(n_mol, box):
    """Lattice dimensions (nx, ny, nz) with nx*ny*nz == n_mol and spacing ~ box/n."""
    vol = box[0] * box[1] * box[2]
    a = (vol / n_mol) ** (1.0 / 3.0)
    dims = tuple(int(round(b / a)) for b in box)
    if dims[0] * dims[1] * dims[2] != n_mol:
        raise ValueError(f"{n_mol} molecules do not fill a {dims} lattice")
    return dims


def make_state(wl: Workload, seed: int | None = None):
    """Return (x, v) for a workload: float64 (3, N_s) each, positions wrapped into the box."""
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    box = wl.box
    n_sites = wl.n_mol * wl.sites_per_mol
    masses = np.tile(np.asarray(wl.site_mass, dtype=np.float64), wl.n_mol)
    if wl.sites_per_mol == 4:
        dims = _lattice_dims(wl.n_mol, box)
        com = lattice_points(dims, box, rng, jitter=0.05)
        x = tetra_positions(com, rng)
    elif wl.sites_per_mol in (2, 3):
        dims = _lattice_dims(wl.n_mol, box)
        com = lattice_points(dims, box, rng, jitter=0.05)
        x = body_positions(com, wl.sites_per_mol, rng)
    elif wl.bond_kind == BOND_FENE:
        n = int(math.ceil(wl.n_mol ** (1.0 / 3.0) - 1e-9))
        path = serpentine_path(n)[: wl.n_mol]
        a = box[0] / n
        x = ((path.T.astype(np.float64) + 0.5) * a)
        x = x + rng.uniform(-0.05 * a, 0.05 * a, size=x.shape)
    else:
        dims = _lattice_dims(wl.n_mol, box)
        x = lattice_points(dims, box, rng, jitter=0.3)
    x = wrap_into_box(x, box)
    v = maxwell_velocities(n_sites, masses, wl.kT, rng)
    return np.ascontiguousarray(x), np.ascontiguousarray(v)


def anchor_molecules(n_mol, k, seed):
    """k distinct molecule indices (sorted): the anchors of a self-adjusting AT region."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_mol, size=k, replace=False)).astype(np.int32)


def random_pair_distances(n, r_lo, r_hi, seed):
    """Uniform random scalar distances, float64 (for pair-function tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(r_lo, r_hi, size=n)


def mlp_init(seed, hidden=64):
    """He-initialised parameters of the 1->H->H->1 CG force network (float64 vector).

    Layout: W1[H], b1[H], W2[H*H] (row = output unit), b2[H], W3[H], b3[1]."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=hidden) * math.sqrt(2.0)
    b1 = rng.uniform(-1.0, 1.0, size=hidden)
    W2 = rng.normal(size=(hidden, hidden)) * math.sqrt(2.0 / hidden)
    b2 = np.zeros(hidden)
    W3 = rng.normal(size=hidden) * math.sqrt(1.0 / hidden)
    b3 = np.zeros(1)
    return np.concatenate([W1, b1, W2.ravel(), b2, W3, b3])


def mlp_n_params(hidden=64):
    return hidden + hidden + hidden * hidden + hidden + hidden + 1
