"""Seeded synthetic inputs for the induced-dipole solve.

The paper benchmarks water boxes of growing size and a solvated protein; none of
those coordinate/parameter sets ship with it, so this module builds stand-ins of
the same shape: rigid waters on a cubic lattice with random orientation and
jitter, a self-avoiding random chain with bonded polarization scalings, and a
sequence of slightly displaced configurations.  It holds no arithmetic of the
method itself (no fields, no Ewald, no solve): only geometry, parameters and
topology, so that both the FP64 oracle and the GPU library consume the same
arrays.

Every array is float64 (int32 for the scaled-pair CSR), in the caller's atom
order.  Units: Angstrom, e, e*A, e*A^2, A^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Rigid water geometry and AMOEBA-like water parameters of the workload recipe.
R_OH = 0.9572
ANG_HOH = np.deg2rad(104.52)
Q_O, Q_H = -0.51966, 0.25983
ALPHA_O, ALPHA_H = 0.837, 0.496
THOLE_A = 0.39
DIPOLE_MAG = 0.1      # e*A
QUAD_SCALE = 0.2      # e*A^2

# Chain solute atom types C/N/O/H and their polarizabilities (A^3).
CHAIN_ALPHA = np.array([1.33, 1.07, 0.84, 0.50])
CHAIN_BOND = 1.5
CHAIN_MIN_NONBONDED = 2.0


@dataclass
class System:
    """One configuration plus its force-field parameters and run settings."""
    name: str
    pos: np.ndarray            # (N,3) A, wrapped into [0, L)
    box: np.ndarray            # (3,) A, orthorhombic
    q: np.ndarray              # (N,) e
    dip: np.ndarray            # (N,3) e*A, lab frame
    quad: np.ndarray           # (N,6) e*A^2 traceless, order xx,xy,xz,yy,yz,zz
    alpha: np.ndarray          # (N,) A^3
    thole: np.ndarray          # (N,) dimensionless Thole a
    sc_ptr: np.ndarray         # (N+1,) int32 CSR row pointers of scaled pairs
    sc_j: np.ndarray           # int32 partner indices (both directions stored)
    sc_s: np.ndarray           # float64 permanent-field scale of each listed pair
    mol: np.ndarray            # (N,) int32 molecule id (chain solute = 0 for C3)
    cutoff: float = 7.0
    buffer: float = 0.0
    ewald_alpha: float = 0.545
    grid: tuple = (24, 24, 24)
    order: int = 5
    tol_debye: float = 1e-5
    seed: int = 0
    meta: dict = field(default_factory=dict)
    sc_s_d: np.ndarray = None  # direct (d) scales of the same CSR pairs (two-set model); None: d = p

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_rotations(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-random rotation matrices from normalised Gaussian quaternions."""
    qv = rng.standard_normal((m, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    r = np.empty((m, 3, 3))
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


def water_template() -> np.ndarray:
    """O at the origin, the two H in the xy plane, bisector along +x."""
    h = ANG_HOH / 2
    return np.array([[0.0, 0.0, 0.0],
                     [R_OH * np.cos(h), R_OH * np.sin(h), 0.0],
                     [R_OH * np.cos(h), -R_OH * np.sin(h), 0.0]])


def random_multipoles(rng: np.random.Generator, n: int):
    """|d| = 0.1 e*A in a uniform direction; Theta = 0.2*(S - tr(S)/3 I), S = sym(G)."""
    v = rng.standard_normal((n, 3))
    dip = DIPOLE_MAG * v / np.linalg.norm(v, axis=1, keepdims=True)
    g = rng.standard_normal((n, 3, 3))
    s = 0.5 * (g + np.transpose(g, (0, 2, 1)))
    tr = np.trace(s, axis1=1, axis2=2) / 3.0
    s -= tr[:, None, None] * np.eye(3)[None]
    s *= QUAD_SCALE
    quad = np.stack([s[:, 0, 0], s[:, 0, 1], s[:, 0, 2], s[:, 1, 1], s[:, 1, 2], s[:, 2, 2]], axis=1)
    quad[:, 5] = -quad[:, 0] - quad[:, 3]       # exact tracelessness in the stored form
    return dip, quad


def build_csr(n: int, pairs: list, scales: list):
    """Symmetric CSR of scaled pairs: every (i, j, s) is stored as i->j and j->i, rows sorted by j."""
    rows = [[] for _ in range(n)]
    for (i, j), s in zip(pairs, scales):
        rows[i].append((j, s))
        rows[j].append((i, s))
    ptr = np.zeros(n + 1, dtype=np.int32)
    js, ss = [], []
    for i in range(n):
        r = sorted(rows[i])
        ptr[i + 1] = ptr[i] + len(r)
        js.extend(j for j, _ in r)
        ss.extend(s for _, s in r)
    return ptr, np.asarray(js, dtype=np.int32), np.asarray(ss, dtype=np.float64)


def _water_csr_arrays(first_atom: int, nw: int):
    """Intramolecular O-H, O-H (1-2) and H-H (1-3) pairs of nw consecutive waters, scale 0."""
    base = first_atom + 3 * np.arange(nw)
    pairs = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1),
                            np.stack([base + 1, base + 2], 1)])
    return pairs, np.zeros(len(pairs))


def _csr_from_arrays(n: int, pairs: np.ndarray, scales: np.ndarray):
    """Vectorised symmetric CSR (rows sorted by partner index)."""
    i = np.concatenate([pairs[:, 0], pairs[:, 1]]).astype(np.int64)
    j = np.concatenate([pairs[:, 1], pairs[:, 0]]).astype(np.int64)
    s = np.concatenate([scales, scales]).astype(np.float64)
    order = np.lexsort((j, i))
    i, j, s = i[order], j[order], s[order]
    counts = np.bincount(i, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(counts)
    return ptr, j.astype(np.int32), s


def place_waters(rng: np.random.Generator, sites: np.ndarray, jitter: float = 0.1) -> np.ndarray:
    """Rigid waters with O at each site + N(0, jitter^2) per axis, Haar-random orientation."""
    m = sites.shape[0]
    rot = random_rotations(rng, m)
    tmpl = water_template()
    centre = sites + jitter * rng.standard_normal((m, 3))
    xyz = centre[:, None, :] + np.einsum('mab,kb->mka', rot, tmpl)
    return xyz.reshape(-1, 3)


def lattice_sites(n_edge: int, box_len: float) -> np.ndarray:
    g = (np.arange(n_edge) + 0.5) * (box_len / n_edge)
    x, y, z = np.meshgrid(g, g, g, indexing='ij')
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1)


def water_box(n_waters: int, box_len: float, grid: int, seed: int, name: str,
              buffer: float = 0.0, tol: float = 1e-5) -> System:
    """Waters on the smallest n^3 lattice holding n_waters; a seeded choice of occupied sites."""
    rng = _rng(seed)
    n_edge = int(np.ceil(round(n_waters ** (1.0 / 3.0), 9)))
    while n_edge ** 3 < n_waters:
        n_edge += 1
    sites = lattice_sites(n_edge, box_len)
    if sites.shape[0] > n_waters:
        keep = np.sort(rng.choice(sites.shape[0], n_waters, replace=False))
        sites = sites[keep]
    pos = place_waters(rng, sites)
    n = pos.shape[0]
    pos = np.mod(pos, box_len)
    q = np.tile([Q_O, Q_H, Q_H], n_waters).astype(np.float64)
    alpha = np.tile([ALPHA_O, ALPHA_H, ALPHA_H], n_waters).astype(np.float64)
    thole = np.full(n, THOLE_A)
    dip, quad = random_multipoles(rng, n)
    pairs, scales = _water_csr_arrays(0, n_waters)
    ptr, sj, ss = _csr_from_arrays(n, pairs, scales)
    mol = np.repeat(np.arange(n_waters, dtype=np.int32), 3)
    return System(name=name, pos=pos, box=np.full(3, float(box_len)), q=q, dip=dip, quad=quad,
                  alpha=alpha, thole=thole, sc_ptr=ptr, sc_j=sj, sc_s=ss, mol=mol,
                  buffer=buffer, grid=(grid, grid, grid), tol_debye=tol, seed=seed,
                  meta={"lattice_edge": n_edge, "n_waters": n_waters, "spacing": box_len / n_edge})


def _min_image(d: np.ndarray, box_len: float) -> np.ndarray:
    return d - box_len * np.round(d / box_len)


def chain_solute(n_chain: int, box_len: float, rng: np.random.Generator) -> np.ndarray:
    """Self-avoiding random walk, 1.5 A bonds, no atom within 2.0 A of an earlier non-bonded atom."""
    pos = np.empty((n_chain, 3))
    pos[0] = 0.5 * box_len
    for i in range(1, n_chain):
        for _ in range(10000):
            v = rng.standard_normal(3)
            cand = pos[i - 1] + CHAIN_BOND * v / np.linalg.norm(v)
            if i >= 2:
                d = _min_image(pos[:i - 1] - cand, box_len)
                if np.min(np.einsum('ij,ij->i', d, d)) < CHAIN_MIN_NONBONDED ** 2:
                    continue
            pos[i] = cand
            break
        else:
            raise RuntimeError("self-avoiding walk got stuck")
    return np.mod(pos, box_len)


def solvated_chain(seed: int = 3, box_len: float = 62.23, n_chain: int = 2489, n_w: int = 7023,
                   lattice: int = 20, grid: int = 64, name: str = "solvated_chain_23558") -> System:
    """2,489-atom chain + 7,023 waters = 23,558 atoms in a 62.23 A box, PME grid 64^3 (the
    defaults); other sizes for tests.  Polarization groups for the direct (d) scales: chain atoms
    3g, 3g+1, 3g+2 form group g (d = 0 inside a group, 1 otherwise), a water is one group."""
    rng = _rng(seed)
    chain = chain_solute(n_chain, box_len, rng)
    types = rng.integers(0, 4, n_chain)
    q_chain = rng.uniform(-0.5, 0.5, n_chain)
    q_chain -= q_chain.mean()
    sites = lattice_sites(lattice, box_len)
    dmin = np.empty(sites.shape[0])
    for s0 in range(0, sites.shape[0], 500):
        d = _min_image(sites[s0:s0 + 500, None, :] - chain[None, :, :], box_len)
        dmin[s0:s0 + 500] = np.sqrt(np.min(np.einsum('abk,abk->ab', d, d), axis=1))
    far = np.argsort(-dmin, kind='stable')[:n_w]
    sites = sites[np.sort(far)]
    wat = place_waters(rng, sites)
    pos = np.mod(np.concatenate([chain, wat]), box_len)
    n = pos.shape[0]
    q = np.concatenate([q_chain, np.tile([Q_O, Q_H, Q_H], n_w)])
    alpha = np.concatenate([CHAIN_ALPHA[types], np.tile([ALPHA_O, ALPHA_H, ALPHA_H], n_w)])
    thole = np.full(n, THOLE_A)
    dip, quad = random_multipoles(rng, n)
    # bonded scalings along the chain: 1-2 and 1-3 excluded, 1-4 halved; water 1-2/1-3 excluded
    ic = np.arange(n_chain)
    p12 = np.stack([ic[:-1], ic[:-1] + 1], 1)
    p13 = np.stack([ic[:-2], ic[:-2] + 2], 1)
    p14 = np.stack([ic[:-3], ic[:-3] + 3], 1)
    wp, ws = _water_csr_arrays(n_chain, n_w)
    pairs = np.concatenate([p12, p13, p14, wp])
    scales = np.concatenate([np.zeros(len(p12)), np.zeros(len(p13)), np.full(len(p14), 0.5), ws])
    ptr, sj, ss = _csr_from_arrays(n, pairs, scales)
    # direct scales of the same pairs: 0 inside a polarization group, 1 between groups
    chain_pairs = np.concatenate([p12, p13, p14])
    d_chain = np.where(chain_pairs[:, 0] // 3 == chain_pairs[:, 1] // 3, 0.0, 1.0)
    _, sj_d, ss_d = _csr_from_arrays(n, pairs, np.concatenate([d_chain, np.zeros(len(wp))]))
    assert np.array_equal(sj_d, sj)
    mol = np.concatenate([np.zeros(n_chain, np.int32), 1 + np.repeat(np.arange(n_w, dtype=np.int32), 3)])
    return System(name=name, pos=pos, box=np.full(3, box_len), q=q, dip=dip, quad=quad,
                  alpha=alpha, thole=thole, sc_ptr=ptr, sc_j=sj, sc_s=ss, mol=mol, buffer=0.0,
                  grid=(grid, grid, grid), tol_debye=1e-5, seed=seed,
                  meta={"n_chain": n_chain, "n_waters": n_w, "types": types.astype(np.int32)}, sc_s_d=ss_d)


def solvated_chain_small(seed: int = 11) -> System:
    """A 240-atom chain + 500 waters (1,740 atoms) in a 26 A box, PME grid 30^3: the two-set
    tests' workload, small enough for the oracle's exact solves."""
    return solvated_chain(seed=seed, box_len=26.0, n_chain=240, n_w=500, lattice=8, grid=30,
                          name="solvated_chain_1740")


def water648(seed: int = 1) -> System:
    """216 waters on a 6^3 lattice in an 18.63 A box, grid 24^3, FP64 to 1e-6 D."""
    return water_box(216, 18.63, 24, seed, "water_648", buffer=0.0, tol=1e-6)


def water96k(seed: int = 2) -> System:
    """32,000 waters (96,000 atoms) in a 98.65 A box, grid 108^3, 2 A list buffer."""
    return water_box(32000, 98.65, 108, seed, "water_96000", buffer=2.0)


def water288k(seed: int = 4) -> System:
    """96,000 waters (288,000 atoms) in a 142.3 A box, grid 144^3, 2 A list buffer."""
    return water_box(96000, 142.3, 144, seed, "water_288000", buffer=2.0)


def water864k(seed: int = 5) -> System:
    """288,000 waters (864,000 atoms) in a 205.0 A box, grid 216^3, 2 A list buffer."""
    return water_box(288000, 205.0, 216, seed, "water_864000", buffer=2.0)


def subcell(parent: System, cells: int = 11, grid: int = 36, seed: int = 6) -> System:
    """A periodic cube cut from a lattice water box: `cells` lattice spacings per edge, whole
    waters whose O lies inside.  Cutting at a whole number of lattice spacings keeps the
    contacts across the new periodic faces at the lattice distance.  The multipoles are
    redrawn from `seed`; geometry and per-molecule parameters are inherited."""
    spacing = parent.meta["spacing"]
    side = cells * spacing
    o_idx = np.arange(0, parent.n, 3)
    o = parent.pos[o_idx]
    inside = np.all(o < side, axis=1)
    mols = np.nonzero(inside)[0]
    atoms = (3 * mols[:, None] + np.arange(3)[None, :]).ravel()
    rng = _rng(seed)
    pos = parent.pos[atoms].copy()
    # unwrap each water around its O, then wrap into the new box
    for k in (1, 2):
        pos[k::3] = pos[0::3] + _min_image(pos[k::3] - pos[0::3], parent.box[0])
    pos = np.mod(pos, side)
    nw = len(mols)
    n = 3 * nw
    dip, quad = random_multipoles(rng, n)
    pairs, scales = _water_csr_arrays(0, nw)
    ptr, sj, ss = _csr_from_arrays(n, pairs, scales)
    return System(name=f"subcell_{n}", pos=pos, box=np.full(3, side), q=parent.q[atoms].copy(), dip=dip,
                  quad=quad, alpha=parent.alpha[atoms].copy(), thole=parent.thole[atoms].copy(),
                  sc_ptr=ptr, sc_j=sj, sc_s=ss, mol=np.repeat(np.arange(nw, dtype=np.int32), 3),
                  buffer=0.0, grid=(grid, grid, grid), tol_debye=1e-5, seed=seed,
                  meta={"n_waters": nw, "parent": parent.name, "side": side})


def trajectory(base: System, n_frames: int, step_sigma: float = 0.02, seed: int = 104):
    """Positions of successive configurations: cumulative per-atom N(0, sigma^2) per axis.
    Frame 0 is the base configuration.  Returns a generator of (N,3) arrays wrapped into the box."""
    rng = _rng(seed)
    cur = base.pos.copy()
    for t in range(n_frames):
        if t > 0:
            cur = cur + step_sigma * rng.standard_normal(cur.shape)
        yield np.mod(cur, base.box)


def guess_init_model(seed: int = 7, n_feat: int = 11, hidden: int = 64, n_basis: int = 3) -> np.ndarray:
    """Starting weights of the learned-guess network as one float32 model vector (layout
    W1[hidden][n_feat], b1, W2[hidden][hidden], b2, W3[n_basis][hidden], b3, mean[n_feat],
    inv_std[n_feat]): W1 and W2 drawn from N(0, 1/fan_in), every other entry zero, so the
    untrained network returns the plain sum of its bases.  The normalisation entries are
    filled by the feature-statistics fit before training."""
    rng = _rng(seed)
    w1 = rng.standard_normal((hidden, n_feat)) / np.sqrt(n_feat)
    w2 = rng.standard_normal((hidden, hidden)) / np.sqrt(hidden)
    parts = [w1.ravel(), np.zeros(hidden), w2.ravel(), np.zeros(hidden), np.zeros(n_basis * hidden),
             np.zeros(n_basis), np.zeros(n_feat), np.ones(n_feat)]
    return np.concatenate(parts).astype(np.float32)


def tiny_cell(n_atoms: int, box_len: float, seed: int, min_dist: float = 0.0,
              with_multipoles: bool = True) -> System:
    """A few atoms at random positions in a small cubic box (rejection keeps them min_dist
    apart under minimum image); neutral charges, random alpha in [0.4, 1.4], Thole 0.39."""
    rng = _rng(seed)
    pos = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place atoms")
        c = rng.uniform(0, box_len, 3)
        if k and min_dist > 0:
            d = _min_image(pos[:k] - c, box_len)
            if np.min(np.linalg.norm(d, axis=1)) < min_dist:
                continue
        pos[k] = c
        k += 1
    q = rng.uniform(-0.5, 0.5, n_atoms)
    q -= q.mean()
    alpha = rng.uniform(0.4, 1.4, n_atoms)
    thole = np.full(n_atoms, THOLE_A)
    if with_multipoles:
        dip, quad = random_multipoles(rng, n_atoms)
    else:
        dip, quad = np.zeros((n_atoms, 3)), np.zeros((n_atoms, 6))
    ptr = np.zeros(n_atoms + 1, np.int32)
    return System(name=f"tiny_{n_atoms}", pos=pos, box=np.full(3, float(box_len)), q=q, dip=dip,
                  quad=quad, alpha=alpha, thole=thole, sc_ptr=ptr, sc_j=np.zeros(0, np.int32),
                  sc_s=np.zeros(0), mol=np.arange(n_atoms, dtype=np.int32), seed=seed)


CONFIGS = {
    "water_648": water648,
    "water_96000": water96k,
    "solvated_chain_23558": solvated_chain,
    "water_288000": water288k,
    "water_864000": water864k,
}


def make(name: str) -> System:
    return CONFIGS[name]()
