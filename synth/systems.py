"""Seeded generators for symmetric, atom-block-sparse Kohn-Sham-like matrices.

Every matrix is returned in the *block-column panel* layout used throughout the
project (host and device):

* ``block_size[a]``   number of orbitals of atom ``a`` (int32)
* ``col_ptr[c]``      CSC pointer over block columns (int64, length n_atoms+1)
* ``row_idx[k]``      block-row (atom) index of stored block ``k``; rows are
                      ascending inside each block column and the diagonal block
                      is always present (int32)
* ``panel_off[c]``    offset of block column ``c``'s *panel* in ``vals`` (int64,
                      length n_atoms+1).  The panel stacks the blocks
                      ``(r, c)`` of the column vertically, in ascending ``r``,
                      into one dense column-major array of height
                      ``h_c = sum_r block_size[r]`` and width ``block_size[c]``.
                      Entry ``(p, q)`` of block ``(r, c)`` sits at
                      ``panel_off[c] + q * h_c + rowoff(r, c) + p``.

The pattern is structurally symmetric and so are the values.  With the
orthogonal basis of every workload here (S = I) the purification formula of the
paper (Eq. 14, P = 1/2 (I - sign(S^-1 H - mu I)) S^-1) reduces to
P = 1/2 (I - sign(H - mu I)).

Readings of the workload descriptions (they are inputs, not the method):

* couplings are drawn once per unordered atom pair i < j (pairs in
  lexicographic order) as a row-major b_i x b_j block B_ij; block (j, i) is
  B_ij^T.  Onsite blocks are diagonal.
* "N(0, s)" is a normal with standard deviation s; "U(a, b)" is uniform.
* one ``numpy.random.default_rng(seed)`` is consumed in this order: vacancies
  (one uniform per lattice site), jitter, molecule positions / orientations,
  couplings (all pairs in one draw), onsite noise (one draw of length N).
* the onsite split that opens a gap: lattice systems put the first b/2
  orbitals of every atom at -split and the rest at +split; water-like systems
  put the first 4 orbitals of every O at -split and every other orbital at
  +split.  The electron count (no spin factor, P = C C^T) is the number of
  "low" orbitals.
* distances use the periodic minimum image.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "BlockSparse", "lattice_system", "water_system", "config1", "config2",
    "config3", "config4", "config5_step", "union", "to_dense",
    "fully_coupled_lattice", "from_pairs", "keyed_normals", "with_onsite_shift",
]


@dataclass
class BlockSparse:
    block_size: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    panel_off: np.ndarray
    vals: np.ndarray
    positions: np.ndarray
    box: float | None
    n_occ: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.block_size.shape[0])

    @property
    def n_orb(self) -> int:
        return int(self.block_size.sum())

    @property
    def nnzb(self) -> int:
        return int(self.row_idx.shape[0])

    @property
    def orb_off(self) -> np.ndarray:
        off = np.zeros(self.n_atoms + 1, dtype=np.int64)
        np.cumsum(self.block_size, out=off[1:])
        return off

    def panel_height(self) -> np.ndarray:
        h = np.zeros(self.n_atoms, dtype=np.int64)
        for c in range(self.n_atoms):
            r = self.row_idx[self.col_ptr[c]:self.col_ptr[c + 1]]
            h[c] = int(self.block_size[r].sum())
        return h

    def with_vals(self, vals: np.ndarray, name: str | None = None) -> "BlockSparse":
        return BlockSparse(self.block_size, self.col_ptr, self.row_idx,
                           self.panel_off, np.ascontiguousarray(vals, dtype=np.float64),
                           self.positions, self.box, self.n_occ,
                           self.name if name is None else name, dict(self.meta))


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _pairs_within(pos: np.ndarray, box: float | None, cutoff: float, chunk: int = 512):
    """All atom pairs i < j with (minimum-image) distance <= cutoff."""
    n = pos.shape[0]
    out_i, out_j, out_r = [], [], []
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = pos[None, :, :] - pos[s:e, None, :]
        if box is not None:
            d -= box * np.round(d / box)
        r = np.sqrt(np.einsum("abk,abk->ab", d, d))
        ii, jj = np.nonzero(r <= cutoff)
        ii = ii + s
        keep = jj > ii
        out_i.append(ii[keep])
        out_j.append(jj[keep])
        out_r.append(r[ii[keep] - s, jj[keep]])
    pi = np.concatenate(out_i).astype(np.int64)
    pj = np.concatenate(out_j).astype(np.int64)
    pr = np.concatenate(out_r)
    order = np.lexsort((pj, pi))
    return pi[order], pj[order], pr[order]


def _assemble(block_size, pi, pj, pair_vals, pair_off, onsite, positions, box,
              n_occ, name, meta):
    """Place pair blocks B_ij (row-major b_i x b_j at pair_off[m]) and the
    diagonal onsite blocks into the block-column panel layout."""
    bs = np.asarray(block_size, dtype=np.int64)
    n = bs.shape[0]
    npair = pi.shape[0]
    rows = np.concatenate([pi, pj, np.arange(n)])
    cols = np.concatenate([pj, pi, np.arange(n)])
    src = np.concatenate([np.arange(npair), np.arange(npair), -np.ones(n, np.int64)])
    kind = np.concatenate([np.zeros(npair, np.int8), np.ones(npair, np.int8),
                           np.full(n, 2, np.int8)])
    order = np.lexsort((rows, cols))
    rows, cols, src, kind = rows[order], cols[order], src[order], kind[order]
    nnzb = rows.shape[0]
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=n), out=col_ptr[1:])
    hb = bs[rows]
    h = np.zeros(n, dtype=np.int64)
    np.add.at(h, cols, hb)
    csum = np.cumsum(hb) - hb
    rowoff = csum - csum[col_ptr[cols]]
    panel_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(h * bs, out=panel_off[1:])
    vals = np.zeros(int(panel_off[-1]), dtype=np.float64)
    orb_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(bs, out=orb_off[1:])

    # diagonal (onsite) blocks: diagonal entries only
    dk = np.nonzero(kind == 2)[0]
    for k in dk:
        c = cols[k]
        b = bs[c]
        p = np.arange(b)
        vals[panel_off[c] + p * h[c] + rowoff[k] + p] = onsite[orb_off[c] + p]

    # off-diagonal blocks, vectorised per (b_r, b_c) shape class
    ok = np.nonzero(kind != 2)[0]
    if ok.size:
        shapes = np.stack([bs[rows[ok]], bs[cols[ok]]], axis=1)
        for br, bc in np.unique(shapes, axis=0):
            sel = ok[(shapes[:, 0] == br) & (shapes[:, 1] == bc)]
            p = np.arange(br)[None, :, None]
            q = np.arange(bc)[None, None, :]
            step = max(1, 4_000_000 // int(br * bc))
            for s in range(0, sel.size, step):
                ks = sel[s:s + step]
                c = cols[ks]
                dest = (panel_off[c] + rowoff[ks])[:, None, None] + p + q * h[c][:, None, None]
                base = pair_off[src[ks]][:, None, None]
                tr = (kind[ks] == 1)[:, None, None]
                # kind 0: block (i, j) = B[p, q] (row-major b_i x b_j)
                # kind 1: block (j, i) = B^T, element (p, q) = B[q, p], B is bc x br
                sidx = np.where(tr, base + q * br + p, base + p * bc + q)
                vals[dest.ravel()] = pair_vals[sidx.ravel()]
    return BlockSparse(block_size=bs.astype(np.int32), col_ptr=col_ptr,
                       row_idx=rows.astype(np.int32), panel_off=panel_off, vals=vals,
                       positions=positions, box=box, n_occ=int(n_occ), name=name,
                       meta=meta)


def _pair_offsets(bs, pi, pj):
    sizes = bs[pi].astype(np.int64) * bs[pj].astype(np.int64)
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off, sizes


# ----------------------------------------------------------------------------
# lattice systems (configurations 1 and 2)
# ----------------------------------------------------------------------------

def lattice_system(n_side: int, n_orb: int, cutoff: float, seed: int = 0, *,
                   spacing: float = 1.0, vacancy: float = 0.0, jitter: float = 0.0,
                   split: float = 1.5, onsite_sigma: float = 0.3, decay: float = 2.0,
                   periodic: bool = True, coupling_cutoff: float | None = None,
                   name: str | None = None) -> BlockSparse:
    """Cubic lattice, n_orb orbitals per atom, couplings -exp(-decay r) U(0.5, 1)
    for atom pairs within ``cutoff``; onsite N(0, onsite_sigma) plus a +/-split
    that puts half of each atom's orbitals low.

    With ``coupling_cutoff`` < ``cutoff`` the pattern still holds every pair
    within ``cutoff`` but pairs farther than ``coupling_cutoff`` store explicit
    zero blocks: the same H on a wider structural pattern (larger index sets)."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side) * spacing
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    if vacancy > 0.0:
        keep = rng.random(sites.shape[0]) >= vacancy
        sites = sites[keep]
    pos = sites.astype(np.float64)
    box = n_side * spacing if periodic else None
    if jitter > 0.0:
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
        if box is not None:
            pos = np.mod(pos, box)
    n = pos.shape[0]
    bs = np.full(n, n_orb, dtype=np.int64)
    pi, pj, pr = _pairs_within(pos, box, cutoff)
    poff, sizes = _pair_offsets(bs, pi, pj)
    u = rng.uniform(0.5, 1.0, size=int(poff[-1]))
    amp = -np.exp(-decay * pr)
    if coupling_cutoff is not None:
        amp = np.where(pr <= coupling_cutoff, amp, 0.0)
    pair_vals = np.repeat(amp, sizes) * u
    nb = n * n_orb
    onsite = rng.normal(0.0, onsite_sigma, size=nb)
    low = np.tile(np.arange(n_orb) < n_orb // 2, n)
    onsite = onsite + np.where(low, -split, split)
    n_occ = int(low.sum())
    meta = dict(kind="lattice", n_side=n_side, n_orb=n_orb, cutoff=cutoff, seed=seed,
                vacancy=vacancy, jitter=jitter, split=split, spacing=spacing,
                coupling_cutoff=coupling_cutoff, atom_ranges=[(0, n)])
    return _assemble(bs, pi, pj, pair_vals, poff, onsite, pos, box, n_occ,
                     name or f"lattice{n_side}_b{n_orb}_rc{cutoff}", meta)


def fully_coupled_lattice(seed: int = 0, n_orb: int = 2) -> BlockSparse:
    """2x2x2 periodic lattice whose cutoff (2.0) exceeds every minimum-image
    distance (at most sqrt 3): every index set is the whole system."""
    return lattice_system(2, n_orb, 2.0, seed, name="fully_coupled_2x2x2")


def config1(seed: int = 0) -> BlockSparse:
    """64 atoms on a periodic 4x4x4 lattice, 4 orbitals, cutoff 1.5 (N = 256)."""
    return lattice_system(4, 4, 1.5, seed, name="cfg1_lattice64")


def config2(seed: int = 0) -> BlockSparse:
    """10x10x10 lattice, 3% vacancies, jitter N(0, 0.05), 6 orbitals,
    cutoff 2.2 (N ~ 5800)."""
    return lattice_system(10, 6, 2.2, seed, vacancy=0.03, jitter=0.05,
                          name="cfg2_lattice1000")


# ----------------------------------------------------------------------------
# water-like systems (configurations 3, 4 and 5)
# ----------------------------------------------------------------------------

_OH = 0.9572 / 3.104          # O-H distance in units of the molecular volume^(1/3)
_HOH = math.radians(104.52)   # H-O-H angle


def _rsa_positions(rng, n_mol, box, min_dist):
    placed = np.empty((n_mol, 3))
    k = 0
    while k < n_mol:
        p = rng.random(3) * box
        if k:
            d = placed[:k] - p
            d -= box * np.round(d / box)
            if np.min(np.einsum("ak,ak->a", d, d)) < min_dist * min_dist:
                continue
        placed[k] = p
        k += 1
    return placed


def _water_geometry(rng, n_mol, density=1.0, min_oo=0.8):
    from scipy.spatial.transform import Rotation
    box = (n_mol / density) ** (1.0 / 3.0)
    o = _rsa_positions(rng, n_mol, box, min_oo)
    rot = Rotation.random(n_mol, random_state=rng).as_matrix()
    s, c = math.sin(_HOH / 2), math.cos(_HOH / 2)
    local = np.array([[0.0, 0.0, 0.0], [_OH * s, 0.0, _OH * c], [-_OH * s, 0.0, _OH * c]])
    pos = o[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    pos = np.mod(pos.reshape(-1, 3), box)
    return pos, box


def _water_block_sizes(n_mol, n_orb_o=13, n_orb_h=5):
    return np.tile(np.array([n_orb_o, n_orb_h, n_orb_h], dtype=np.int64), n_mol)


def _water_onsite(rng, bs, sigma, split, n_low_o=4):
    n_mol = bs.shape[0] // 3
    onsite = rng.normal(0.0, sigma, size=int(bs.sum()))
    low = np.zeros(int(bs.sum()), dtype=bool)
    per = int(bs[:3].sum())
    for m in range(n_mol):
        low[m * per:m * per + n_low_o] = True
    return onsite + np.where(low, -split, split), int(low.sum())


def water_system(n_mol: int, cutoff: float, seed=0, *, density: float = 1.0,
                 min_oo: float = 0.8, decay: float = 1.5, split: float = 6.0,
                 onsite_sigma: float = 0.3, name: str | None = None) -> BlockSparse:
    """n_mol water-like molecules (O with 13 orbitals, two H with 5) placed by
    random sequential addition at the given density; block couplings
    exp(-decay r) N(0, 1) for every atom pair within ``cutoff``."""
    rng = np.random.default_rng(seed)
    pos, box = _water_geometry(rng, n_mol, density, min_oo)
    bs = _water_block_sizes(n_mol)
    pi, pj, pr = _pairs_within(pos, box, cutoff)
    poff, sizes = _pair_offsets(bs, pi, pj)
    g = rng.standard_normal(size=int(poff[-1]))
    pair_vals = np.repeat(np.exp(-decay * pr), sizes) * g
    onsite, n_occ = _water_onsite(rng, bs, onsite_sigma, split)
    meta = dict(kind="water", n_mol=n_mol, cutoff=cutoff, seed=seed, split=split,
                atom_ranges=[(0, 3 * n_mol)])
    return _assemble(bs, pi, pj, pair_vals, poff, onsite, pos, box, n_occ,
                     name or f"water{n_mol}_rc{cutoff}", meta)


def config3(seed: int = 0, n_mol: int = 1000, cutoff: float = 3.0) -> BlockSparse:
    """1000 water-like molecules at density 1, cutoff 3.0 (N = 23000)."""
    return water_system(n_mol, cutoff, seed, name=f"cfg3_water{n_mol}")


CONFIG4_PARTS = ((250, 2.5), (500, 2.5 + 1.0 / 3.0), (1000, 2.5 + 2.0 / 3.0), (2000, 3.5))


def config4(seed: int = 0, parts=CONFIG4_PARTS) -> BlockSparse:
    """Four independent water-like systems (250/500/1000/2000 molecules, cutoffs
    rising with size) as one block-diagonal matrix: one batch, four systems."""
    systems = [water_system(nm, rc, [seed, k], name=f"water{nm}")
               for k, (nm, rc) in enumerate(parts)]
    return union(systems, name="cfg4_mixed_water")


def union(systems, name="union") -> BlockSparse:
    """Block-diagonal union of independent systems (no coupling between them)."""
    bs = np.concatenate([s.block_size.astype(np.int64) for s in systems])
    col_ptr = [np.zeros(1, np.int64)]
    rows, vals, poff = [], [], [np.zeros(1, np.int64)]
    a0, v0, k0 = 0, 0, 0
    ranges = []
    for s in systems:
        rows.append(s.row_idx.astype(np.int64) + a0)
        col_ptr.append(s.col_ptr[1:] + k0)
        poff.append(s.panel_off[1:] + v0)
        vals.append(s.vals)
        ranges.append((a0, a0 + s.n_atoms))
        a0 += s.n_atoms
        k0 += s.nnzb
        v0 += s.vals.shape[0]
    pos = np.concatenate([s.positions for s in systems])
    meta = dict(kind="union", parts=[s.meta for s in systems], atom_ranges=ranges,
                n_occ_parts=[s.n_occ for s in systems])
    return BlockSparse(bs.astype(np.int32), np.concatenate(col_ptr),
                       np.concatenate(rows).astype(np.int32), np.concatenate(poff),
                       np.concatenate(vals), pos, None, sum(s.n_occ for s in systems),
                       name, meta)


# ---- configuration 5: a smooth trajectory of the configuration-3 system ----

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def keyed_normals(seed: int, i: np.ndarray, j: np.ndarray, count: np.ndarray) -> np.ndarray:
    """Standard normals keyed by (seed, i, j, element): the same pair always
    gets the same block, whichever step it appears in (Box-Muller on two
    SplitMix64 uniforms)."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    count = np.asarray(count, dtype=np.int64)
    key = _splitmix64(_splitmix64(_splitmix64(np.full(i.shape, seed, np.uint64)) ^ i) ^ j)
    kk = np.repeat(key, count)
    start = np.zeros(count.shape[0] + 1, dtype=np.int64)
    np.cumsum(count, out=start[1:])
    e = (np.arange(int(start[-1]), dtype=np.int64) - np.repeat(start[:-1], count)).astype(np.uint64)
    with np.errstate(over="ignore"):
        a = _splitmix64(kk ^ (e * np.uint64(2)))
        b = _splitmix64(kk ^ (e * np.uint64(2) + np.uint64(1)))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def config5_step(step: int, seed: int = 0, n_mol: int = 1000, cutoff: float = 3.0,
                 sigma: float = 0.02) -> BlockSparse:
    """Geometry ``step`` (0 = start) of a random walk of the configuration-3
    system: every atom moves by N(0, sigma) per step; coupling factors and
    onsite noise are fixed per atom pair / orbital, so H changes smoothly."""
    rng = np.random.default_rng(seed)
    pos, box = _water_geometry(rng, n_mol)
    bs = _water_block_sizes(n_mol)
    onsite, n_occ = _water_onsite(np.random.default_rng([seed, 1]), bs, 0.3, 6.0)
    for s in range(1, step + 1):
        pos = pos + np.random.default_rng([seed, 5, s]).normal(0.0, sigma, size=pos.shape)
    pos = np.mod(pos, box)
    pi, pj, pr = _pairs_within(pos, box, cutoff)
    poff, sizes = _pair_offsets(bs, pi, pj)
    g = keyed_normals(seed, pi, pj, sizes)
    pair_vals = np.repeat(np.exp(-1.5 * pr), sizes) * g
    meta = dict(kind="water_traj", n_mol=n_mol, cutoff=cutoff, seed=seed, step=step,
                split=6.0, atom_ranges=[(0, 3 * n_mol)])
    return _assemble(bs, pi, pj, pair_vals, poff, onsite, pos, box, n_occ,
                     f"cfg5_water{n_mol}_step{step}", meta)


# ----------------------------------------------------------------------------
# layout conversion (small systems only)
# ----------------------------------------------------------------------------

def to_dense(m: BlockSparse) -> np.ndarray:
    """Dense N x N copy of a block-column-panel matrix (layout only)."""
    off = m.orb_off
    n = int(off[-1])
    out = np.zeros((n, n))
    for c in range(m.n_atoms):
        rs = m.row_idx[m.col_ptr[c]:m.col_ptr[c + 1]]
        h = int(m.block_size[rs].sum())
        bc = int(m.block_size[c])
        panel = m.vals[m.panel_off[c]:m.panel_off[c] + h * bc].reshape(bc, h).T
        ro = 0
        for r in rs:
            br = int(m.block_size[r])
            out[off[r]:off[r] + br, off[c]:off[c] + bc] = panel[ro:ro + br]
            ro += br
    return out


def from_pairs(block_size, pairs, blocks, onsite, n_occ, name="custom") -> BlockSparse:
    """Build a matrix from explicit pair blocks: ``pairs`` is a list of (i, j)
    with i < j and ``blocks[m]`` the b_i x b_j block of pair m; ``onsite`` is the
    diagonal of the onsite blocks (length N)."""
    bs = np.asarray(block_size, dtype=np.int64)
    pi = np.array([p[0] for p in pairs], dtype=np.int64)
    pj = np.array([p[1] for p in pairs], dtype=np.int64)
    if pi.size:
        order = np.lexsort((pj, pi))
        pi, pj = pi[order], pj[order]
        blocks = [np.asarray(blocks[k], dtype=np.float64) for k in order]
    poff, _ = _pair_offsets(bs, pi, pj)
    flat = np.concatenate([b.ravel() for b in blocks]) if pi.size else np.zeros(0)
    pos = np.zeros((bs.shape[0], 3))
    return _assemble(bs, pi, pj, flat, poff, np.asarray(onsite, dtype=np.float64), pos,
                     None, n_occ, name, dict(kind="custom", atom_ranges=[(0, bs.shape[0])]))


def with_onsite_shift(m: BlockSparse, atom: int, orbital: int, shift: float) -> BlockSparse:
    """A copy of ``m`` with ``shift`` added to the diagonal entry of one orbital
    (an isolated state far from the rest of the spectrum, e.g. +20 on one
    orbital of a lattice system: it stretches the Gershgorin bracket and the
    spectral radius of every submatrix that contains the atom)."""
    rows = m.row_idx[m.col_ptr[atom]:m.col_ptr[atom + 1]]
    h = int(m.block_size[rows].sum())
    loc = int(m.block_size[rows[rows < atom]].sum())
    vals = m.vals.copy()
    vals[m.panel_off[atom] + orbital * h + loc + orbital] += shift
    return m.with_vals(vals, name=f"{m.name}+shift({atom},{orbital},{shift:g})")


# ----------------------------------------------------------------------------
# overlap matrices (non-orthogonal basis)
# ----------------------------------------------------------------------------

def overlap_for(m: BlockSparse, seed: int = 0, strength: float = 0.5, decay: float = 2.0,
                max_row_sum: float = 0.6) -> BlockSparse:
    """A synthetic overlap matrix S on the same block pattern as ``m``:
    identity onsite blocks, pair blocks strength * exp(-decay r) * U(-0.2, 1)
    (r the minimum-image distance of the two atoms), symmetric.  If the
    largest off-diagonal absolute row sum exceeds ``max_row_sum`` all pair
    blocks are scaled down to it, so every eigenvalue of S (and of every
    principal submatrix) lies in [1 - max_row_sum, 1 + max_row_sum]."""
    rng = np.random.default_rng([seed, 0x5EED])
    bs = np.asarray(m.block_size, dtype=np.int64)
    cols = np.repeat(np.arange(m.n_atoms), np.diff(m.col_ptr))
    rows = np.asarray(m.row_idx, dtype=np.int64)
    keep = rows < cols
    pi, pj = rows[keep], cols[keep]
    order = np.lexsort((pj, pi))
    pi, pj = pi[order], pj[order]
    d = m.positions[pj] - m.positions[pi]
    if m.box is not None:
        d -= m.box * np.round(d / m.box)
    r = np.sqrt((d ** 2).sum(1))
    poff, sizes = _pair_offsets(bs, pi, pj)
    vals = rng.uniform(-0.2, 1.0, size=int(poff[-1])) * np.repeat(strength * np.exp(-decay * r), sizes)
    # largest absolute row sum over the pair blocks (rows of i from B_ij, of j from B_ij^T)
    rs = np.zeros(int(bs.sum()))
    off = np.zeros(m.n_atoms + 1, dtype=np.int64)
    np.cumsum(bs, out=off[1:])
    for k in range(pi.shape[0]):
        B = np.abs(vals[poff[k]:poff[k + 1]]).reshape(bs[pi[k]], bs[pj[k]])
        rs[off[pi[k]]:off[pi[k] + 1]] += B.sum(1)
        rs[off[pj[k]]:off[pj[k] + 1]] += B.sum(0)
    top = float(rs.max()) if rs.size else 0.0
    if top > max_row_sum:
        vals *= max_row_sum / top
    return _assemble(bs, pi, pj, vals, poff, np.ones(int(bs.sum())), m.positions, m.box, m.n_occ,
                     f"{m.name}:S", dict(m.meta, overlap_seed=seed))
