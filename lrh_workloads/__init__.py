"""Seeded synthetic problem generators shared by the oracle and the GPU path.

This module only *describes* problems: sites, local Hamiltonian terms on their
supports, the top-level cluster family and the instance each site belongs to.
It holds none of the relaxation's arithmetic (no poset, no lifting, no
eigen-decomposition of augmented Hamiltonians, no message updates).

Conventions (the paper leaves them open, so they are fixed here):
  * spin-1/2 sites, Pauli matrices X, Y, Z (no factor 1/2);
  * a term on sites (s_0 < s_1 < ...) is a dense matrix in the big-endian
    product basis of those sites, i.e. A_{s0} (x) B_{s1} == np.kron(A, B);
  * the Hamiltonian is H = sum_e h_e + sum_v h_v with every term stored on its
    own support (Sec. 3.1 of the paper, 2-local form).

A problem is the plain-array `ProblemDesc` below; it mirrors the C struct the
library takes, so both sides consume byte-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import math

import numpy as np

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


@dataclass
class ProblemDesc:
    """Plain-array description of H = sum of local terms plus a cluster family."""

    name: str
    n_sites: int
    site_dim: np.ndarray            # int32 [n_sites]
    term_ptr: np.ndarray            # int64 [n_terms+1], CSR over term_sites
    term_sites: np.ndarray          # int32, ascending within each term
    term_off: np.ndarray            # int64 [n_terms+1], offsets into term_re/term_im
    term_re: np.ndarray             # float64, row-major dense blocks
    term_im: Optional[np.ndarray]   # float64 or None when every term is real
    top_ptr: np.ndarray             # int64 [n_top+1]
    top_sites: np.ndarray           # int32, ascending within each cluster
    site_instance: np.ndarray       # int32 [n_sites]
    n_instances: int
    subintervals: bool = False      # add every contiguous run of each top cluster
    two_level: bool = False         # family = top clusters + their maximal pairwise overlaps
    # Optional linear parametrisation of terms, h_t = sum_p c_p * B_{t,p}; used by
    # gradient workloads.  term_param[t] = index of the coupling the term is
    # proportional to (-1: constant term), dterm_* = d h_t / d c.
    term_param: Optional[np.ndarray] = None
    params: Optional[np.ndarray] = None
    dterm_re: Optional[np.ndarray] = None
    dterm_im: Optional[np.ndarray] = None
    meta: Dict = field(default_factory=dict)

    @property
    def n_terms(self) -> int:
        return len(self.term_ptr) - 1

    @property
    def n_top(self) -> int:
        return len(self.top_ptr) - 1

    @property
    def is_real(self) -> bool:
        return self.term_im is None

    def term(self, t: int) -> Tuple[Tuple[int, ...], np.ndarray]:
        sites = tuple(int(s) for s in self.term_sites[self.term_ptr[t]:self.term_ptr[t + 1]])
        D = int(np.prod([self.site_dim[s] for s in sites]))
        a, b = self.term_off[t], self.term_off[t + 1]
        m = self.term_re[a:b].reshape(D, D).astype(np.complex128)
        if self.term_im is not None:
            m = m + 1j * self.term_im[a:b].reshape(D, D)
        return sites, m

    def terms(self) -> Iterable[Tuple[Tuple[int, ...], np.ndarray]]:
        for t in range(self.n_terms):
            yield self.term(t)

    def dterm(self, t: int) -> Optional[np.ndarray]:
        if self.dterm_re is None:
            return None
        a, b = self.term_off[t], self.term_off[t + 1]
        D = int(round(np.sqrt(b - a)))
        m = self.dterm_re[a:b].reshape(D, D).astype(np.complex128)
        if self.dterm_im is not None:
            m = m + 1j * self.dterm_im[a:b].reshape(D, D)
        return m

    def top(self, c: int) -> Tuple[int, ...]:
        return tuple(int(s) for s in self.top_sites[self.top_ptr[c]:self.top_ptr[c + 1]])

    def tops(self) -> Iterable[Tuple[int, ...]]:
        for c in range(self.n_top):
            yield self.top(c)


# --------------------------------------------------------------------------------------
# assembly helpers (input bookkeeping only)
# --------------------------------------------------------------------------------------

def _reorder(sites: Sequence[int], mat: np.ndarray, dims: Sequence[int]):
    """Return (sorted sites, matrix with tensor factors permuted to that order)."""
    sites = list(sites)
    order = sorted(range(len(sites)), key=lambda i: sites[i])
    if order == list(range(len(sites))):
        return tuple(sites), mat
    k = len(sites)
    d = [dims[i] for i in range(k)]
    t = mat.reshape(d + d)
    t = t.transpose(order + [k + o for o in order])
    D = int(np.prod(d))
    return tuple(sites[i] for i in order), t.reshape(D, D)


class _Builder:
    def __init__(self, name: str, n_sites: int, d: int = 2):
        self.name = name
        self.n = n_sites
        self.site_dim = np.full(n_sites, d, dtype=np.int32)
        self.terms: List[Tuple[Tuple[int, ...], np.ndarray, int, Optional[np.ndarray]]] = []
        self.tops: List[Tuple[int, ...]] = []
        self.site_instance = np.zeros(n_sites, dtype=np.int32)
        self.n_instances = 1

    def add_term(self, sites, mat, param: int = -1, dmat=None):
        dims = [int(self.site_dim[s]) for s in sites]
        if len(set(sites)) != len(sites):
            raise ValueError("term support has repeated sites")
        s2, m2 = _reorder(sites, np.asarray(mat, dtype=np.complex128), dims)
        d2 = None
        if dmat is not None:
            _, d2 = _reorder(sites, np.asarray(dmat, dtype=np.complex128), dims)
        self.terms.append((s2, m2, param, d2))

    def add_top(self, sites):
        s = tuple(sorted(int(x) for x in sites))
        if len(set(s)) != len(s):
            raise ValueError("cluster has repeated sites")
        self.tops.append(s)

    def build(self, real: Optional[bool] = None, subintervals=False, params=None, meta=None,
              two_level=False):
        n_t = len(self.terms)
        term_ptr = np.zeros(n_t + 1, dtype=np.int64)
        term_off = np.zeros(n_t + 1, dtype=np.int64)
        for t, (s, m, _, _) in enumerate(self.terms):
            term_ptr[t + 1] = term_ptr[t] + len(s)
            term_off[t + 1] = term_off[t] + m.size
        term_sites = np.array([x for (s, _, _, _) in self.terms for x in s], dtype=np.int32)
        flat = (np.concatenate([m.reshape(-1) for (_, m, _, _) in self.terms])
                if n_t else np.zeros(0, np.complex128))
        if real is None:
            real = bool(np.all(flat.imag == 0))
        term_re = np.ascontiguousarray(flat.real, dtype=np.float64)
        term_im = None if real else np.ascontiguousarray(flat.imag, dtype=np.float64)
        if real and np.any(flat.imag != 0):
            raise ValueError("real storage requested for a complex term")
        term_param = None
        dre = dim = None
        if any(p >= 0 for (_, _, p, _) in self.terms):
            term_param = np.array([p for (_, _, p, _) in self.terms], dtype=np.int32)
            dflat = np.concatenate([
                (dm if dm is not None else np.zeros_like(m)).reshape(-1)
                for (_, m, _, dm) in self.terms])
            dre = np.ascontiguousarray(dflat.real)
            dim = None if real else np.ascontiguousarray(dflat.imag)
        top_ptr = np.zeros(len(self.tops) + 1, dtype=np.int64)
        for c, s in enumerate(self.tops):
            top_ptr[c + 1] = top_ptr[c] + len(s)
        top_sites = np.array([x for s in self.tops for x in s], dtype=np.int32)
        return ProblemDesc(
            name=self.name, n_sites=self.n, site_dim=self.site_dim.copy(),
            term_ptr=term_ptr, term_sites=term_sites, term_off=term_off,
            term_re=term_re, term_im=term_im, top_ptr=top_ptr, top_sites=top_sites,
            site_instance=self.site_instance.copy(), n_instances=self.n_instances,
            subintervals=subintervals, two_level=bool(two_level), term_param=term_param,
            params=None if params is None else np.asarray(params, dtype=np.float64),
            dterm_re=dre, dterm_im=dim, meta=dict(meta or {}))


def kron(*ms):
    out = np.array([[1.0 + 0j]])
    for m in ms:
        out = np.kron(out, m)
    return out


def gue(rng: np.random.Generator, D: int) -> np.ndarray:
    """A D x D draw from the Gaussian unitary ensemble: (G + G^H)/2, G complex Ginibre."""
    g = rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D))
    return (g + g.conj().T) / 2


# --------------------------------------------------------------------------------------
# model Hamiltonians
# --------------------------------------------------------------------------------------

def tfim_chain(n: int, J: float = 1.0, h: float = 0.5, complex_storage: bool = True,
               field_on_sites: bool = True) -> ProblemDesc:
    """Open transverse-field Ising chain H = -J sum Z_i Z_{i+1} - h sum X_i.

    Cluster family: the edges (i, i+1); singletons are added by the relaxation.
    """
    b = _Builder(f"tfim_chain_n{n}", n)
    for i in range(n - 1):
        b.add_term((i, i + 1), -J * kron(Z, Z))
        b.add_top((i, i + 1))
    if field_on_sites:
        for i in range(n):
            b.add_term((i,), -h * X)
    else:
        # field folded into the edges: X_0 fully on edge 0, X_{n-1} on the last edge,
        # interior sites split evenly between their two edges.
        for i in range(n - 1):
            wi = 1.0 if i == 0 else 0.5
            wj = 1.0 if i + 1 == n - 1 else 0.5
            b.add_term((i, i + 1), -h * (wi * kron(X, I2) + wj * kron(I2, X)))
    return b.build(real=not complex_storage, meta=dict(model="tfim", J=J, h=h, n=n))


def heisenberg_graph(n: int, edges: Sequence[Tuple[int, int]], J: float = 1.0,
                     name: str = "heisenberg", field_x: float = 0.0) -> ProblemDesc:
    """H = J sum_(ij) (X X + Y Y + Z Z) + field_x sum X_i on an arbitrary graph."""
    b = _Builder(name, n)
    hxx = (kron(X, X) + kron(Y, Y) + kron(Z, Z)) * J
    for (i, j) in edges:
        b.add_term((i, j), hxx)
        b.add_top((i, j))
    if field_x != 0.0:
        for i in range(n):
            b.add_term((i,), field_x * X)
    return b.build(real=True, meta=dict(model="heisenberg", J=J, edges=len(edges)))


def square_edges(L: int, periodic: bool = True, offset: int = 0):
    edges = []
    for y in range(L):
        for x in range(L):
            s = offset + x + L * y
            if periodic or x + 1 < L:
                edges.append((s, offset + (x + 1) % L + L * y))
            if periodic or y + 1 < L:
                edges.append((s, offset + x + L * ((y + 1) % L)))
    return edges


def heisenberg_square(L: int = 32, J: float = 1.0) -> ProblemDesc:
    """Heisenberg antiferromagnet on the L x L periodic square lattice (site x + L y)."""
    if L < 3:
        raise ValueError("periodic square lattice needs L >= 3")
    return heisenberg_graph(L * L, square_edges(L), J, name=f"heisenberg_square_L{L}")


def heisenberg_chain(n: int, J: float = 1.0, field_x: float = 0.0) -> ProblemDesc:
    return heisenberg_graph(n, [(i, i + 1) for i in range(n - 1)], J,
                            name=f"heisenberg_chain_n{n}", field_x=field_x)


def anisotropic_heisenberg_chain(n: int, Jx: float = 2.0, Jy: float = -3.0, Jz: float = 0.5,
                                 field_x: float = 0.0):
    b = _Builder(f"xyz_chain_n{n}" + (f"_hx{field_x:g}" if field_x else ""), n)
    hh = Jx * kron(X, X) + Jy * kron(Y, Y) + Jz * kron(Z, Z)
    for i in range(n - 1):
        b.add_term((i, i + 1), hh)
        b.add_top((i, i + 1))
    if field_x:
        for i in range(n):
            b.add_term((i,), field_x * X)
    return b.build(real=True, meta=dict(model="xyz", J=(Jx, Jy, Jz), field_x=field_x))


def random_chain(n: int, seed: int, scale: float = 1.0, top_len: int = 2,
                 subintervals: bool = False, two_level: bool = False) -> ProblemDesc:
    """Chain with independent GUE 2-site terms; top clusters are intervals of length top_len."""
    rng = np.random.default_rng(seed)
    b = _Builder(f"random_chain_n{n}_s{seed}", n)
    for i in range(n - 1):
        b.add_term((i, i + 1), scale * gue(rng, 4))
    for i in range(n - top_len + 1):
        b.add_top(tuple(range(i, i + top_len)))
    return b.build(real=False, subintervals=subintervals, two_level=two_level,
                   meta=dict(model="random", seed=seed, top_len=top_len))


def interval_chain_gue(n: int, k: int, eps: float = 0.1, seed: int = 3, two_level: bool = False) -> ProblemDesc:
    """Weakly perturbed separable chain of Thm. 3: H = sum h_i + eps sum v_{i,i+1}.

    h_i = V_i diag(0, 1) V_i^H with V_i the eigenvectors of a seeded 2x2 GUE draw
    (unit norm, unique ground state of energy 0, gap 1); v_{i,i+1} is a 4x4 GUE draw
    scaled to spectral norm 1.  Draw order: every h_i first, then every v_i.
    Cluster family: the interval hierarchy Y_k (all intervals of length k and every
    contiguous sub-interval), or with two_level=True only the windows of length k and the
    overlaps of consecutive windows (the same optimum on a chain).
    """
    rng = np.random.default_rng(seed)
    b = _Builder(f"interval_chain_n{n}_k{k}_s{seed}", n)
    for i in range(n):
        w, V = np.linalg.eigh(gue(rng, 2))
        b.add_term((i,), V @ np.diag([0.0, 1.0]) @ V.conj().T)
    for i in range(n - 1):
        v = gue(rng, 4)
        v = v / np.max(np.abs(np.linalg.eigvalsh(v)))
        b.add_term((i, i + 1), eps * v)
    for i in range(n - k + 1):
        b.add_top(tuple(range(i, i + k)))
    return b.build(real=False, subintervals=not two_level, two_level=two_level,
                   meta=dict(model="interval_gue", eps=eps, seed=seed, k=k, n=n, two_level=two_level))


SQ2 = np.sqrt(0.5)
SX1 = SQ2 * np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=np.complex128)
SY1 = SQ2 * np.array([[0, -1j, 0], [1j, 0, -1j], [0, 1j, 0]], dtype=np.complex128)
SZ1 = np.diag([1.0, 0.0, -1.0]).astype(np.complex128)


def spin1_chain(n: int, J: float = 1.0, Dz: float = 0.3, hx: float = 0.2, dm: float = 0.0,
                top_len: int = 2, subintervals: bool = False, two_level: bool = False) -> ProblemDesc:
    """Open spin-1 chain (site dimension 3): H = J sum S_i . S_{i+1} + Dz sum (S^z_i)^2
    + hx sum S^x_i + dm sum (S^x_i S^y_{i+1} - S^y_i S^x_{i+1}).  The last (Dzyaloshinskii-Moriya)
    term is imaginary in the S^z basis, so dm != 0 gives a complex problem.  Top clusters: the
    windows of top_len consecutive sites (with subintervals: the interval hierarchy Y_top_len)."""
    b = _Builder(f"spin1_chain_n{n}_t{top_len}", n, d=3)
    bond = J * (kron(SX1, SX1) + kron(SY1, SY1) + kron(SZ1, SZ1))
    if dm != 0.0:
        bond = bond + dm * (kron(SX1, SY1) - kron(SY1, SX1))
    for i in range(n - 1):
        b.add_term((i, i + 1), bond)
    for i in range(n):
        b.add_term((i,), Dz * SZ1 @ SZ1 + hx * SX1)
    for i in range(n - top_len + 1):
        b.add_top(tuple(range(i, i + top_len)))
    return b.build(real=(dm == 0.0), subintervals=subintervals, two_level=two_level,
                   meta=dict(model="spin1_chain", n=n, J=J, Dz=Dz, hx=hx, dm=dm, top_len=top_len))


def tfim_plaquette_batch(Ls: Sequence[int], hs: Sequence[float], J: float = 1.0,
                         name: str = "tfim_plaquette_batch", two_level: bool = False) -> ProblemDesc:
    """Independent periodic L x L TFIM instances, H_b = -J sum ZZ - h_b sum X.

    Cluster family per instance: every 2x2 plaquette {(x,y),(x+1,y),(x,y+1),(x+1,y+1)} (with
    two_level=True the plaquettes and the bonds they share only).
    Sites of instance b are numbered offset_b + x + L y.
    """
    n = int(sum(L * L for L in Ls))
    b = _Builder(name, n)
    off = 0
    zz = -J * kron(Z, Z)
    for inst, (L, h) in enumerate(zip(Ls, hs)):
        if L < 3:
            raise ValueError("periodic plaquettes need L >= 3")
        L = int(L)
        b.site_instance[off:off + L * L] = inst
        for (i, j) in square_edges(L, True, off):
            b.add_term((i, j), zz)
        for s in range(off, off + L * L):
            b.add_term((s,), -h * X)
        for y in range(L):
            for x in range(L):
                sid = lambda xx, yy: off + (xx % L) + L * (yy % L)
                b.add_top((sid(x, y), sid(x + 1, y), sid(x, y + 1), sid(x + 1, y + 1)))
        off += L * L
    b.n_instances = len(Ls)
    return b.build(real=True, two_level=two_level,
                   meta=dict(model="tfim_plaquette", Ls=list(map(int, Ls)), hs=list(map(float, hs)), J=J))


def tfim_rect_plaquettes(L: int, h: float, w: int = 2, hgt: int = 3, J: float = 1.0) -> ProblemDesc:
    """Periodic L x L TFIM with w x hgt rectangular plaquettes as top clusters (2 x 3: six sites,
    64-dimensional clusters; the interior bonds of a plaquette become its children)."""
    n = L * L
    b = _Builder(f"tfim_rect{w}x{hgt}_L{L}", n)
    zz = -J * kron(Z, Z)
    for (i, j) in square_edges(L, True, 0):
        b.add_term((i, j), zz)
    for s_ in range(n):
        b.add_term((s_,), -h * X)
    sid = lambda xx, yy: (xx % L) + L * (yy % L)
    for y in range(L):
        for x in range(L):
            b.add_top(tuple(sid(x + dx, y + dy) for dy in range(hgt) for dx in range(w)))
    return b.build(real=True, meta=dict(model="tfim_rect", L=L, h=h, w=w, hgt=hgt))


def tfim_growing_clusters(L: int, h: float, level: int = 1, J: float = 1.0) -> ProblemDesc:
    """Periodic L x L TFIM (H = -J sum ZZ - h sum X) on a growing-cluster hierarchy (Sec. 3.2):
    level 0 is the 2 x 2 plaquette family C, level 1 is C plus every 2 x 3 and 3 x 2 rectangle
    (C_{+1}: each rectangle covers two plaquettes, its children in the poset).  L >= 4, so that no
    rectangle wraps onto itself."""
    if L < 4:
        raise ValueError("the rectangles need L >= 4")
    n = L * L
    b = _Builder(f"tfim_grow{level}_L{L}", n)
    zz = -J * kron(Z, Z)
    for (i, j) in square_edges(L, True, 0):
        b.add_term((i, j), zz)
    for s_ in range(n):
        b.add_term((s_,), -h * X)
    sid = lambda xx, yy: (xx % L) + L * (yy % L)
    shapes = [(2, 2)] + ([(3, 2), (2, 3)] if level >= 1 else [])
    for (w, hgt) in shapes:
        for y in range(L):
            for x in range(L):
                b.add_top(tuple(sorted(sid(x + dx, y + dy) for dy in range(hgt) for dx in range(w))))
    return b.build(real=True, meta=dict(model="tfim_growing", L=L, h=h, level=level))


def tfim_plaquette_sweep(n_inst: int = 512, seed: int = 4, Lmin: int = 8, Lmax: int = 64,
                         two_level: bool = False):
    """The batched sweep: L ~ U{Lmin..Lmax}, h ~ U[0.5, 4], drawn in that order."""
    rng = np.random.default_rng(seed)
    Ls = rng.integers(Lmin, Lmax + 1, n_inst)
    hs = rng.uniform(0.5, 4.0, n_inst)
    return tfim_plaquette_batch(Ls, hs, name=f"tfim_plaquette_sweep_{n_inst}_s{seed}", two_level=two_level)


def triangular_edges(L: int):
    """Edges of the L x L periodic triangular lattice in the canonical order:
    for each site (x, y) (site id x + L y, y-major), the bonds to (x+1,y), (x,y+1), (x+1,y+1)."""
    sid = lambda x, y: (x % L) + L * (y % L)
    edges = []
    for y in range(L):
        for x in range(L):
            edges.append((sid(x, y), sid(x + 1, y)))
            edges.append((sid(x, y), sid(x, y + 1)))
            edges.append((sid(x, y), sid(x + 1, y + 1)))
    return edges


def xxz_triangular(L: int = 64, Delta: float = 0.5, seed: int = 5, n_bonds: int = 32,
                   Jlo: float = 0.8, Jhi: float = 1.2, two_level: bool = False) -> ProblemDesc:
    """XXZ model J_e (XX + YY + Delta ZZ) on the periodic triangular lattice with up and
    down triangles as clusters.  J_e ~ U[Jlo, Jhi] in canonical edge order; then
    `n_bonds` distinct bonds are drawn for gradient checks (meta['bonds']).  two_level=True:
    the triangles and their overlaps (the bonds) only, each bond term split over its two
    triangles."""
    if L < 3:
        raise ValueError("triangular lattice needs L >= 3")
    rng = np.random.default_rng(seed)
    edges = triangular_edges(L)
    J = rng.uniform(Jlo, Jhi, len(edges))
    bonds = rng.choice(len(edges), min(n_bonds, len(edges)), replace=False)
    b = _Builder(f"xxz_triangular_L{L}_s{seed}", L * L)
    B = kron(X, X) + kron(Y, Y) + Delta * kron(Z, Z)
    for e, (i, j) in enumerate(edges):
        b.add_term((i, j), J[e] * B, param=e, dmat=B)
    sid = lambda x, y: (x % L) + L * (y % L)
    for y in range(L):
        for x in range(L):
            b.add_top((sid(x, y), sid(x + 1, y), sid(x + 1, y + 1)))
            b.add_top((sid(x, y), sid(x, y + 1), sid(x + 1, y + 1)))
    return b.build(real=True, params=J, two_level=two_level,
                   meta=dict(model="xxz_triangular", L=L, Delta=Delta, seed=seed,
                             bonds=[int(x) for x in bonds]))


def classical_ising_tree(n: int, seed: int, rotate: bool = False) -> ProblemDesc:
    """Diagonal Ising model J_ij Z_i Z_j + h_i Z_i on a random tree (J, h ~ U[-1, 1]).

    The tree attaches site i to a uniformly drawn earlier site.  With rotate=True every
    site is conjugated by a seeded Haar-random unitary U_i: the terms stay commuting
    but are no longer diagonal.
    """
    rng = np.random.default_rng(seed)
    parent = [int(rng.integers(0, i)) for i in range(1, n)]
    Js = rng.uniform(-1, 1, n - 1)
    hs = rng.uniform(-1, 1, n)
    Us = []
    for _ in range(n):
        if rotate:
            g = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
            q, r = np.linalg.qr(g)
            Us.append(q * (np.diag(r) / np.abs(np.diag(r))))
        else:
            Us.append(I2)
    b = _Builder(f"ising_tree_n{n}_s{seed}{'_rot' if rotate else ''}", n)
    for i in range(1, n):
        p = parent[i - 1]
        a, c = min(p, i), max(p, i)
        U = np.kron(Us[a], Us[c])
        b.add_term((a, c), U @ (Js[i - 1] * kron(Z, Z)) @ U.conj().T)
        b.add_top((a, c))
    for i in range(n):
        b.add_term((i,), Us[i] @ (hs[i] * Z) @ Us[i].conj().T)
    return b.build(real=not rotate,
                   meta=dict(model="ising_tree", parent=parent, J=Js.tolist(), h=hs.tolist(),
                             rotate=rotate))


def whole_system(desc: ProblemDesc) -> ProblemDesc:
    """The same terms with one top cluster holding every site (the relaxation is then exact)."""
    b = _Builder(desc.name + "_whole", desc.n_sites)
    b.site_dim = desc.site_dim.copy()
    for s, m in desc.terms():
        b.add_term(s, m)
    b.add_top(tuple(range(desc.n_sites)))
    return b.build(real=desc.is_real)


def with_tops(desc: ProblemDesc, tops: Sequence[Sequence[int]], subintervals=False,
              name: Optional[str] = None, two_level: bool = False) -> ProblemDesc:
    """Same terms, another top-level cluster family."""
    b = _Builder(name or desc.name + "_tops", desc.n_sites)
    b.site_dim = desc.site_dim.copy()
    b.site_instance = desc.site_instance.copy()
    b.n_instances = desc.n_instances
    for s, m in desc.terms():
        b.add_term(s, m)
    for t in tops:
        b.add_top(t)
    return b.build(real=desc.is_real, subintervals=subintervals, two_level=two_level)


# --------------------------------------------------------------------------------------
# seeded message draws (keyed by the cluster pair, so both sides draw identical values
# whatever order they enumerate messages in)
# --------------------------------------------------------------------------------------

def batch_scaled(descs: Sequence[ProblemDesc], scales: Sequence[float], name: str = "batch") -> ProblemDesc:
    """Independent instances in one problem: instance i is descs[i] with every term multiplied
    by scales[i] (sites renumbered, top clusters kept).  Parametrised terms are not carried."""
    n = int(sum(d.n_sites for d in descs))
    b = _Builder(name, n)
    off = 0
    subint = None
    for i, (d, sc) in enumerate(zip(descs, scales)):
        if subint is None:
            subint = (d.subintervals, d.two_level)
        elif subint != (d.subintervals, d.two_level):
            raise ValueError("instances disagree on the cluster family")
        b.site_dim[off:off + d.n_sites] = d.site_dim
        b.site_instance[off:off + d.n_sites] = i
        for sites, m in d.terms():
            b.add_term(tuple(off + x for x in sites), float(sc) * m)
        for t in d.tops():
            b.add_top(tuple(off + x for x in t))
        off += d.n_sites
    b.n_instances = len(descs)
    real = all(d.is_real for d in descs)
    return b.build(real=real, subintervals=bool(subint[0]), two_level=bool(subint[1]),
                   meta=dict(model="batch", scales=list(map(float, scales))))


def message_draw(seed: int, parent: Sequence[int], child: Sequence[int], D: int,
                 real: bool, scale: float = 1.0) -> np.ndarray:
    """A seeded Hermitian (real symmetric when real=True) D x D matrix for message parent->child."""
    ss = np.random.SeedSequence([int(seed), len(parent), *map(int, parent), *map(int, child)])
    rng = np.random.default_rng(ss)
    a = rng.normal(size=(D, D))
    if real:
        m = (a + a.T) / 2
        return (scale * m).astype(np.complex128)
    b = rng.normal(size=(D, D))
    g = a + 1j * b
    return scale * (g + g.conj().T) / 2


# --------------------------------------------------------------------------------------
# the five benchmark workloads
# --------------------------------------------------------------------------------------

def workload_c1() -> ProblemDesc:
    """Level-1 TFIM open chain n=16, J=1, h=0.5, complex storage (subgradient, FP64)."""
    return tfim_chain(16, 1.0, 0.5, complex_storage=True)


def workload_c2(L: int = 32) -> ProblemDesc:
    """Level-1 Heisenberg antiferromagnet on the 32x32 periodic square lattice (real)."""
    return heisenberg_square(L)


def workload_c3(k: int, n: int = 4096, eps: float = 0.1, seed: int = 3, two_level: bool = False) -> ProblemDesc:
    return interval_chain_gue(n, k, eps, seed, two_level=two_level)


def workload_c4(n_inst: int = 512, seed: int = 4, Lmin: int = 8, Lmax: int = 64,
                two_level: bool = False) -> ProblemDesc:
    return tfim_plaquette_sweep(n_inst, seed, Lmin, Lmax, two_level=two_level)


def workload_c5(L: int = 64, seed: int = 5) -> ProblemDesc:
    return xxz_triangular(L, 0.5, seed)


def exact_spectrum_matrix(lam, cplx: bool = False) -> np.ndarray:
    """(H/sqrt(D)) diag(lam) (H/sqrt(D)) with H the Sylvester Hadamard matrix and lam integers:
    every entry is a multiple of 1/D (exact in FP64) and the spectrum is exactly lam.  cplx:
    conjugated by diag(i^k), which multiplies entries by powers of i (exact as well)."""
    D = len(lam)
    H = np.array([[1.0]])
    while H.shape[0] < D:
        H = np.block([[H, H], [H, -H]])
    if H.shape[0] != D:
        raise ValueError("D must be a power of two")
    A = (H @ np.diag(np.asarray(lam, np.float64)) @ H) / D
    if not np.array_equal(A * D, np.round(A * D)):
        raise ValueError("entries not exact: integers too large")
    if cplx:
        s = np.array([1j ** k for k in range(D)])
        A = (s[:, None] * A) * np.conj(s)[None, :]
    return A


def exact_spectrum_problem(lam, cplx: bool = False) -> ProblemDesc:
    """One term on log2(D) qubits whose matrix has exactly the spectrum lam (integers)."""
    D = len(lam)
    k = int(round(math.log2(D)))
    b = _Builder(f"exact_spectrum_{D}", k)
    b.add_term(tuple(range(k)), exact_spectrum_matrix(lam, cplx))
    return b.build(real=not cplx)
