"""Plain FP64 CPU oracle for the local-relaxation message-passing dual.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path (the HIP library and
its binding) never imports, links or executes anything under oracle/, and this
module imports nothing from the product path: the two share only the seeded
problem generators in lrh_workloads.

What is computed (paper, Sec. 4 "Distributed algorithm"):
  * cluster family C_full = top clusters, every term support, every singleton,
    and (interval hierarchy Y_t, eq. interval_set_defn) every contiguous run of
    each top cluster;  the poset keeps only covering relations (Sec. 4.2: only
    constraints between consecutive poset levels are needed);
  * local augmented Hamiltonian (Sec. 4.2, definition of theta_e)
        theta_e = h_e - sum_{f child of e} 1_{e\\f} (x) nu_{e->f} + sum_{g parent of e} nu_{g->e};
  * non-smooth dual Q(nu) = sum_e lambda_min(theta_e)     (eq. dual_function_non-smooth,
    and its cluster form Q_C);
  * soft minimum F_beta(H) = lambda_1 - (1/beta) log sum_k exp(-beta (lambda_k - lambda_1))
    (Sec. 4.1.2 and the stable form in the proof of the smoothing-error lemma);
  * gradient of the smoothed dual: rho_f - Tr_{e\\f} rho_e with rho the Gibbs states
    (Sec. 4.1.2 / 4.2.2);
  * subgradient: mu_f - Tr_{e\\f} mu_e with mu a ground state (Sec. 4.1.1 / 4.2.1);
  * Algorithm 1 (constant/variable-step subgradient ascent with best-iterate tracking)
    and Algorithm 2 (accelerated ascent on the smoothed dual).

Readings where the paper is silent or inconsistent:
  * sign convention: the expanded Lagrangian of Sec. 4.1 (edge Hamiltonian gets
    -nu (x) 1, node Hamiltonian +nu, ascent nu += alpha (mu_i - Tr_j mu_ij));
  * "a sampled zero-energy eigenvector" is read as the normalised ground-space
    projector P0/g, g the multiplicity of eigenvalues within tau of lambda_min,
    tau = 1e-9 * max(1, ||theta_e||_F);
  * basis convention: sites of a cluster in ascending order, first site most
    significant (A_{s0} (x) B_{s1} == np.kron(A, B));
  * every message update is followed by Hermitian symmetrisation (nu + nu^H)/2;
  * Lipschitz constant: L = beta (Delta_G + d)/2 when C_full only has edges and
    sites (Lemma "Lipschitz constant of the smoothed dual"), else
    L = beta Lambda_G / 2 with Lambda_G = max_{e->f} (m_f + m_e D_e / D_f) (Sec. 4.2.2);
  * beta continuation (not in the paper): each stage restarts Algorithm 2 from the
    current nu with zeta = nu, theta = 1;
  * certified value: Q(nu) minus the rounding margin sum_e 8 D_e eps_64 ||theta_e||_F.
"""
from __future__ import annotations

import math
from itertools import combinations
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

EPS64 = np.finfo(np.float64).eps


# --------------------------------------------------------------------------------------
# lift and partial trace (batched over a leading axis; plain einsum on the tensor form)
# --------------------------------------------------------------------------------------

def _axes(dims_e: Sequence[int], pos: Sequence[int]):
    k = len(dims_e)
    rest = [i for i in range(k) if i not in pos]
    Df = int(np.prod([dims_e[i] for i in pos])) if pos else 1
    Dr = int(np.prod([dims_e[i] for i in rest])) if rest else 1
    return list(pos), rest, Df, Dr


def lift(X: np.ndarray, dims_e: Sequence[int], pos: Sequence[int]) -> np.ndarray:
    """1_{e\\f} (x) X written in e's site order.  X: (..., Df, Df), f's sites sit at
    positions `pos` (ascending) of e's sorted site list with local dims `dims_e`."""
    pos, rest, Df, Dr = _axes(dims_e, pos)
    k = len(dims_e)
    batch = X.shape[:-2]
    full = np.einsum('...ab,rs->...arbs', X, np.eye(Dr))          # (f, rest) x (f, rest)
    order = pos + rest
    t = full.reshape(batch + tuple(dims_e[i] for i in order) * 2)
    inv = np.argsort(order)
    nb = len(batch)
    perm = list(range(nb)) + [nb + int(i) for i in inv] + [nb + k + int(i) for i in inv]
    De = int(np.prod(dims_e))
    return t.transpose(perm).reshape(batch + (De, De))


def ptrace(A: np.ndarray, dims_e: Sequence[int], pos: Sequence[int]) -> np.ndarray:
    """Tr_{e\\f} A, keeping the sites at positions `pos` (ascending) of e."""
    pos, rest, Df, Dr = _axes(dims_e, pos)
    k = len(dims_e)
    batch = A.shape[:-2]
    nb = len(batch)
    t = A.reshape(batch + tuple(dims_e) * 2)
    order = pos + rest
    perm = list(range(nb)) + [nb + i for i in order] + [nb + k + i for i in order]
    t = t.transpose(perm).reshape(batch + (Df, Dr, Df, Dr))
    return np.einsum('...arbr->...ab', t)


def herm(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))


# --------------------------------------------------------------------------------------
# the relaxation: poset, augmented Hamiltonians, dual values and (sub)gradients
# --------------------------------------------------------------------------------------

def maximal_overlaps(tops: Sequence[Tuple[int, ...]]) -> List[Tuple[int, ...]]:
    """Non-empty intersections of two top clusters that no other such intersection strictly
    contains.  For the windows of length t on a chain these are the n - t overlaps of
    consecutive windows (length t - 1)."""
    holders: Dict[int, List[int]] = {}
    for i, c in enumerate(tops):
        for v in c:
            holders.setdefault(v, []).append(i)
    inter = set()
    for hs in holders.values():          # only pairs that share a site intersect
        for a, b in combinations(hs, 2):
            inter.add(tuple(sorted(set(tops[a]) & set(tops[b]))))
    # an intersection strictly inside another one shares a site with it
    by_site: Dict[int, List[Tuple[int, ...]]] = {}
    for c in inter:
        for v in c:
            by_site.setdefault(v, []).append(c)
    return sorted(c for c in inter if not any(set(c) < set(o) for o in by_site[c[0]]))


class Relaxation:
    """Cluster poset of one problem (all instances) and the dual's building blocks."""

    def __init__(self, desc, Lambda: Optional[float] = None, herm_tol: float = 1e-12):
        self.desc = desc
        n = desc.n_sites
        sd = [int(x) for x in desc.site_dim]
        self.site_dim = sd
        terms = list(desc.terms())
        self.two_level = bool(getattr(desc, "two_level", False))
        if self.two_level and desc.subintervals:
            raise ValueError("the two-level family and the interval closure exclude each other")
        # ---- C_full (Sec. 3.2 cluster family; Y_t adds contiguous runs) -------------
        cset = set()
        if self.two_level:
            # top clusters and the maximal pairwise overlaps of top clusters, nothing else
            tops = sorted(set(desc.tops()))
            cset.update(tops)
            cset.update(maximal_overlaps(tops))
        else:
            for top in desc.tops():
                cset.add(top)
                if desc.subintervals:
                    for a in range(len(top)):
                        for b in range(a + 1, len(top) + 1):
                            cset.add(top[a:b])
            for s, _ in terms:
                cset.add(s)
            for v in range(n):
                cset.add((v,))
        self.clusters: List[Tuple[int, ...]] = sorted(cset, key=lambda c: (len(c), c))
        self.index: Dict[Tuple[int, ...], int] = {c: i for i, c in enumerate(self.clusters)}
        nc = len(self.clusters)
        self.D = np.array([int(np.prod([sd[s] for s in c])) for c in self.clusters], dtype=np.int64)
        inst = desc.site_instance
        self.inst = np.empty(nc, dtype=np.int64)
        for i, c in enumerate(self.clusters):
            ii = {int(inst[s]) for s in c}
            if len(ii) != 1:
                raise ValueError(f"cluster {c} spans instances {ii}")
            self.inst[i] = ii.pop()
        self.n_inst = int(desc.n_instances)
        # ---- Hasse diagram: maximal proper subsets present in C_full -----------------
        self.children: List[List[int]] = [[] for _ in range(nc)]
        self.parents: List[List[int]] = [[] for _ in range(nc)]
        for e, c in enumerate(self.clusters):
            k = len(c)
            subs = []
            for r in range(k - 1, 0, -1):
                for comb in combinations(c, r):
                    if comb in self.index:
                        subs.append(comb)
            maximal = [f for f in subs if not any(set(f) < set(g) for g in subs)]
            self.children[e] = sorted(self.index[f] for f in maximal)
        for e in range(nc):
            for f in self.children[e]:
                self.parents[f].append(e)
        # ---- messages (one per covering pair e -> f) -------------------------------
        self.msgs: List[Tuple[int, int]] = [(e, f) for e in range(nc) for f in self.children[e]]
        self.msg_index = {m: i for i, m in enumerate(self.msgs)}
        # ---- h_e ---------------------------------------------------------------------
        # closure family: the sum of the terms whose support is exactly e;
        # two-level family: every term split evenly over the top clusters holding its
        # support, lifted into each (same primal objective wherever the tops agree on
        # the term's support)
        self.term_homes: List[List[Tuple[int, Tuple[int, ...], float]]] = []
        if self.two_level:
            holders: Dict[int, List[int]] = {}
            for c in tops:
                for v in c:
                    holders.setdefault(v, []).append(self.index[c])
        for s, m in terms:
            if not np.allclose(m, m.conj().T, atol=herm_tol * max(1.0, np.abs(m).max())):
                raise ValueError(f"term on {s} is not Hermitian")
            if self.two_level:
                homes = [e for e in holders.get(s[0], []) if set(s) <= set(self.clusters[e])]
                if not homes:
                    raise ValueError(f"term on {s} lies in no top cluster")
                w = 1.0 / len(homes)
                self.term_homes.append([(e, tuple(self.clusters[e].index(v) for v in s), w)
                                        for e in homes])
            else:
                e = self.index[s]
                self.term_homes.append([(e, tuple(range(len(s))), 1.0)])
        self.h: Dict[int, np.ndarray] = {}
        for (s, m), homes in zip(terms, self.term_homes):
            for e, pos, w in homes:
                dims_e = [sd[v] for v in self.clusters[e]]
                self.h[e] = self.h.get(e, 0) + w * lift(m, dims_e, pos)
        self.real = desc.is_real
        # ---- groups for batched evaluation ---------------------------------------
        self.cgroups: Dict[int, np.ndarray] = {}
        for D in sorted(set(self.D.tolist())):
            self.cgroups[D] = np.nonzero(self.D == D)[0]
        self.cslot = np.empty(nc, dtype=np.int64)
        for D, ids in self.cgroups.items():
            self.cslot[ids] = np.arange(len(ids))
        # message storage: per child dimension Df, an array (M_Df, Df, Df)
        self.mDf = np.array([self.D[f] for (_, f) in self.msgs], dtype=np.int64)
        self.mslot = np.empty(len(self.msgs), dtype=np.int64)
        self.mgroups_by_Df: Dict[int, np.ndarray] = {}
        for Df in sorted(set(self.mDf.tolist())):
            ids = np.nonzero(self.mDf == Df)[0]
            self.mgroups_by_Df[Df] = ids
            self.mslot[ids] = np.arange(len(ids))
        # patterns: messages sharing (dims_e, pos) use one einsum
        pats: Dict[Tuple, List[int]] = {}
        for m, (e, f) in enumerate(self.msgs):
            ce, cf = self.clusters[e], self.clusters[f]
            pos = tuple(ce.index(s) for s in cf)
            dims_e = tuple(sd[s] for s in ce)
            pats.setdefault((dims_e, pos), []).append(m)
        self.patterns = {k: np.array(v, dtype=np.int64) for k, v in pats.items()}
        self.Lambda = self._lambda() if Lambda is None else float(Lambda)
        self.Gamma = float(np.sum(np.log(self.D)))

    # ---- sizes -------------------------------------------------------------------
    @property
    def n_clusters(self):
        return len(self.clusters)

    @property
    def n_msgs(self):
        return len(self.msgs)

    def _lambda(self) -> float:
        two_local = all(len(c) <= 2 for c in self.clusters)
        if two_local:
            # Lemma (Lipschitz constant of the smoothed dual): Delta_G + d
            deg = max((len(self.parents[e]) for e in range(self.n_clusters)
                       if len(self.clusters[e]) == 1), default=0)
            return float(deg + max(self.site_dim))
        lam = 0.0
        m_ = [len(self.parents[e]) + len(self.children[e]) for e in range(self.n_clusters)]
        for (e, f) in self.msgs:
            lam = max(lam, m_[f] + m_[e] * self.D[e] / self.D[f])
        return float(lam)

    def Delta_G(self) -> int:
        return max((len(self.parents[e]) for e in range(self.n_clusters)
                    if len(self.clusters[e]) == 1), default=0)

    # ---- message containers -----------------------------------------------------
    def zeros(self) -> Dict[int, np.ndarray]:
        return {Df: np.zeros((len(ids), Df, Df), dtype=np.complex128)
                for Df, ids in self.mgroups_by_Df.items()}

    def get(self, nu, m: int) -> np.ndarray:
        return nu[int(self.mDf[m])][self.mslot[m]]

    def set(self, nu, m: int, X: np.ndarray):
        nu[int(self.mDf[m])][self.mslot[m]] = X

    def from_pairs(self, mats: Dict[Tuple[Tuple[int, ...], Tuple[int, ...]], np.ndarray]):
        nu = self.zeros()
        for m, (e, f) in enumerate(self.msgs):
            self.set(nu, m, mats[(self.clusters[e], self.clusters[f])])
        return nu

    def to_pairs(self, nu):
        return {(self.clusters[e], self.clusters[f]): self.get(nu, m).copy()
                for m, (e, f) in enumerate(self.msgs)}

    def draw(self, seed: int, scale: float = 1.0):
        """Seeded messages keyed by cluster pair (identical on every side)."""
        from lrh_workloads import message_draw
        nu = self.zeros()
        for m, (e, f) in enumerate(self.msgs):
            self.set(nu, m, message_draw(seed, self.clusters[e], self.clusters[f],
                                         int(self.D[f]), self.real, scale))
        return nu

    # ---- theta_e (definition of the local augmented Hamiltonian) -----------------
    def thetas(self, nu, with_h: bool = True, h=None) -> Dict[int, np.ndarray]:
        """theta_e for every cluster; with_h=False gives the linear part (B nu)_e alone."""
        hh = self.h if h is None else h
        th = {}
        for D, ids in self.cgroups.items():
            t = np.zeros((len(ids), D, D), dtype=np.complex128)
            if with_h:
                for j, e in enumerate(ids):
                    if int(e) in hh:
                        t[j] = hh[int(e)]
            th[D] = t
        for (dims_e, pos), ms in self.patterns.items():
            De = int(np.prod(dims_e))
            es = np.array([self.msgs[m][0] for m in ms])
            fs = np.array([self.msgs[m][1] for m in ms])
            Df = int(self.D[fs[0]])
            X = nu[Df][self.mslot[ms]]
            np.subtract.at(th[De], self.cslot[es], lift(X, dims_e, pos))   # child messages
            np.add.at(th[Df], self.cslot[fs], X)                            # parent messages
        return th

    def theta(self, nu, e: int) -> np.ndarray:
        """theta_e for one cluster, written out term by term."""
        c = self.clusters[e]
        t = np.array(self.h.get(e, np.zeros((self.D[e], self.D[e]))), dtype=np.complex128)
        for f in self.children[e]:
            pos = tuple(c.index(s) for s in self.clusters[f])
            t = t - lift(self.get(nu, self.msg_index[(e, f)]), [self.site_dim[s] for s in c], pos)
        for g in self.parents[e]:
            t = t + self.get(nu, self.msg_index[(g, e)])
        return t

    # ---- per-instance sums ----------------------------------------------------------
    def _per_instance(self, vals: Dict[int, np.ndarray]) -> np.ndarray:
        out = [[] for _ in range(self.n_inst)]
        for D, ids in self.cgroups.items():
            for j, e in enumerate(ids):
                out[self.inst[e]].append(float(vals[D][j]))
        return np.array([math.fsum(v) for v in out])

    # ---- Q(nu): non-smooth dual -----------------------------------------------------
    def lambda_min(self, nu) -> Dict[int, np.ndarray]:
        th = self.thetas(nu)
        return {D: np.linalg.eigvalsh(t)[:, 0] for D, t in th.items()}

    def Q(self, nu) -> np.ndarray:
        return self._per_instance(self.lambda_min(nu))

    # ---- Q_beta(nu) and its gradient ------------------------------------------------
    def gibbs(self, nu, beta: float):
        """Per cluster: (F_beta, rho_beta).  Stable form lambda_1 - log(sum e^{-b(l-l1)})/b."""
        th = self.thetas(nu)
        F, rho = {}, {}
        for D, t in th.items():
            lam, U = np.linalg.eigh(t)
            w = np.exp(-beta * (lam - lam[:, :1]))
            Zs = w.sum(axis=1)
            F[D] = lam[:, 0] - np.log(Zs) / beta
            p = w / Zs[:, None]
            rho[D] = herm(np.einsum('nik,nk,njk->nij', U, p, U.conj()))
        return F, rho

    def Q_beta(self, nu, beta: float) -> np.ndarray:
        F, _ = self.gibbs(nu, beta)
        return self._per_instance(F)

    def _grad_from_marginals(self, marg) -> Dict[int, np.ndarray]:
        g = self.zeros()
        for (dims_e, pos), ms in self.patterns.items():
            De = int(np.prod(dims_e))
            es = np.array([self.msgs[m][0] for m in ms])
            fs = np.array([self.msgs[m][1] for m in ms])
            Df = int(self.D[fs[0]])
            g[Df][self.mslot[ms]] = marg[Df][self.cslot[fs]] - ptrace(marg[De][self.cslot[es]], dims_e, pos)
        return g

    def grad_beta(self, nu, beta: float):
        """(Q_beta per instance, gradient rho_f - Tr_{e\\f} rho_e for every message)."""
        F, rho = self.gibbs(nu, beta)
        return self._per_instance(F), self._grad_from_marginals(rho)

    # ---- ground projectors and subgradient ------------------------------------------
    def ground(self, nu, tau_rel: float = 1e-9):
        th = self.thetas(nu)
        lmin, mu = {}, {}
        for D, t in th.items():
            lam, U = np.linalg.eigh(t)
            tau = tau_rel * np.maximum(1.0, np.linalg.norm(t, axis=(1, 2)))
            sel = (lam <= lam[:, :1] + tau[:, None]).astype(np.float64)
            g = sel.sum(axis=1)
            lmin[D] = lam[:, 0]
            mu[D] = herm(np.einsum('nik,nk,njk->nij', U, sel / g[:, None], U.conj()))
        return lmin, mu

    def subgrad(self, nu, tau_rel: float = 1e-9):
        lmin, mu = self.ground(nu, tau_rel)
        return self._per_instance(lmin), self._grad_from_marginals(mu)

    # ---- certified bound --------------------------------------------------------------
    def certify(self, nu):
        """(Q(nu), margin) per instance; Q - margin is the reported certified bound."""
        th = self.thetas(nu)
        lm, mg = {}, {}
        for D, t in th.items():
            lm[D] = np.linalg.eigvalsh(t)[:, 0]
            mg[D] = 8.0 * D * EPS64 * np.linalg.norm(t, axis=(1, 2))
        return self._per_instance(lm), self._per_instance(mg)

    # ---- message arithmetic helpers -------------------------------------------------
    @staticmethod
    def axpby(a, x, b, y):
        return {k: a * x[k] + b * y[k] for k in x}

    @staticmethod
    def copy(x):
        return {k: v.copy() for k, v in x.items()}

    @staticmethod
    def symmetrise(x):
        return {k: herm(v) for k, v in x.items()}

    def msg_instance(self) -> Dict[int, np.ndarray]:
        return {Df: self.inst[np.array([self.msgs[m][0] for m in ids])]
                for Df, ids in self.mgroups_by_Df.items()}

    def lipschitz(self, beta: float) -> float:
        return beta * self.Lambda / 2.0


# --------------------------------------------------------------------------------------
# Algorithm 1: subgradient ascent with best-iterate tracking
# --------------------------------------------------------------------------------------

def subgradient(R: Relaxation, T: int, step=None, nu0=None, record_every: int = 0,
                tau_rel: float = 1e-9):
    """Algorithm 1.  step(k) gives alpha_k (k 0-indexed); default 1/sqrt(k+1).

    q^k = Q(nu^k) is evaluated before the update; the best iterate is tracked per
    instance.  Returns (nu_best, q_best, nu_T, history of q^k)."""
    if step is None:
        step = lambda k: 1.0 / math.sqrt(k + 1.0)
    nu = R.zeros() if nu0 is None else R.copy(nu0)
    q_best = np.full(R.n_inst, -np.inf)
    nu_best = R.copy(nu)
    minst = R.msg_instance()
    hist = []
    for k in range(T):
        q, g = R.subgrad(nu, tau_rel)
        hist.append(q)
        better = q > q_best
        if np.any(better):
            q_best = np.where(better, q, q_best)
            for Df in nu:
                sel = better[minst[Df]]
                nu_best[Df][sel] = nu[Df][sel]
        a = step(k)
        nu = R.symmetrise({Df: nu[Df] + a * g[Df] for Df in nu})
    return nu_best, q_best, nu, np.array(hist)


# --------------------------------------------------------------------------------------
# Algorithm 2: accelerated ascent on the smoothed dual, with beta continuation
# --------------------------------------------------------------------------------------

def theta_next(th: float) -> float:
    return (math.sqrt(th ** 4 + 4 * th ** 2) - th ** 2) / 2.0


def nesterov(R: Relaxation, schedule: Sequence[Tuple[float, int]], nu0=None,
             callback=None):
    """Algorithm 2 run stage by stage.  `schedule` lists (beta, iterations); every stage
    starts from the current nu with zeta = nu and theta = 1 (the first stage is exactly
    Algorithm 2's initialisation nu = zeta = 0, theta_0 = 1).  callback(k_global, nu) is
    called after every update."""
    nu = R.zeros() if nu0 is None else R.copy(nu0)
    kg = 0
    for beta, K in schedule:
        L = R.lipschitz(beta)
        zeta = R.copy(nu)
        th = 1.0
        for _ in range(int(K)):
            eta = R.axpby(1.0 - th, nu, th, zeta)
            _, g = R.grad_beta(eta, beta)
            zeta = R.symmetrise({k: zeta[k] + g[k] / (th * L) for k in zeta})
            nu = R.symmetrise(R.axpby(1.0 - th, nu, th, zeta))
            th = theta_next(th)
            kg += 1
            if callback is not None:
                callback(kg, nu)
    return nu


def doubling_schedule(beta0: float, beta_max: float, total_iters: int):
    """beta = beta0 * 2^s up to beta_max, total_iters split evenly, remainder to the last stage."""
    betas = []
    b = beta0
    while b <= beta_max * (1 + 1e-12):
        betas.append(b)
        b *= 2
    per = total_iters // len(betas)
    sched = [(bb, per) for bb in betas]
    sched[-1] = (betas[-1], total_iters - per * (len(betas) - 1))
    return sched


# --------------------------------------------------------------------------------------
# adjoint of the smoothed dual (used by gradient checks)
# --------------------------------------------------------------------------------------

def gibbs_vjp(theta: np.ndarray, beta: float, rho_bar: np.ndarray) -> np.ndarray:
    """theta_bar = d<rho_beta(theta), rho_bar>/d theta for one Hermitian theta.

    With theta = U diag(l) U^H, p = softmax(-beta l): the derivative of rho = U diag(p) U^H
    is the Daleckii-Krein divided-difference formula of the matrix function
    f(x) = exp(-beta x) followed by normalisation:
        theta_bar = U [Gamma o (U^H rho_bar U)] U^H + beta <rho, rho_bar> rho,
    Gamma_ab = (p_a - p_b)/(l_a - l_b) (a != b),  Gamma_aa = -beta p_a.
    (The sign: d rho = U[Gamma o (U^H E U)]U^H + beta <rho, E> rho for theta -> theta + E.)
    (Daleckii-Krein is textbook matrix calculus, not from the paper.)"""
    lam, U = np.linalg.eigh(theta)
    w = np.exp(-beta * (lam - lam[0]))
    p = w / w.sum()
    D = len(lam)
    G = np.empty((D, D))
    for a in range(D):
        for b in range(D):
            # (p_a - p_b)/(l_a - l_b) = p_lo * expm1(-beta (l_hi - l_lo)) / (l_hi - l_lo) with
            # lo the lower eigenvalue: no cancellation, limit -beta p_a when l_a == l_b.
            hi, lo = (a, b) if lam[a] >= lam[b] else (b, a)
            dl = lam[hi] - lam[lo]
            if dl == 0.0:
                G[a, b] = -beta * p[lo]
            else:
                G[a, b] = p[lo] * np.expm1(-beta * dl) / dl
    rho = (U * p) @ U.conj().T
    M = U.conj().T @ rho_bar @ U
    out = U @ (G * M) @ U.conj().T + beta * np.real(np.vdot(rho, rho_bar)) * rho
    return herm(out)


# --------------------------------------------------------------------------------------
# parametrised terms and reverse mode (gradient checks of the certified bound)
# --------------------------------------------------------------------------------------

def term_params(R: Relaxation):
    """[(cluster id, parameter index, d h_t / d c)] for every parametrised term."""
    d = R.desc
    out = []
    if d.term_param is None:
        return out
    for t in range(d.n_terms):
        p = int(d.term_param[t])
        if p >= 0:
            B = d.dterm(t)
            for e, pos, w in R.term_homes[t]:
                dims_e = [R.site_dim[v] for v in R.clusters[e]]
                out.append((e, p, w * lift(B, dims_e, pos)))
    return out


def h_at_params(R: Relaxation, params) -> Dict[int, np.ndarray]:
    """h_e with every parametrised term h_t = c_p * dh_t/dc moved to the new parameters."""
    h = {e: v.copy() for e, v in R.h.items()}
    c0 = R.desc.params
    for e, p, B in term_params(R):
        h[e] = h[e] + (params[p] - c0[p]) * B
    return h


def gibbs_vjp_batch(theta: np.ndarray, beta: float, Xbar: np.ndarray) -> np.ndarray:
    """gibbs_vjp over a stack of clusters (the same formula with a leading batch axis)."""
    lam, U = np.linalg.eigh(theta)
    w = np.exp(-beta * (lam - lam[:, :1]))
    p = w / w.sum(axis=1, keepdims=True)
    la, lb = lam[:, :, None], lam[:, None, :]
    p_lo = np.where(la <= lb, p[:, :, None], p[:, None, :])
    dl = np.abs(la - lb)
    safe = np.where(dl == 0.0, 1.0, dl)
    G = np.where(dl == 0.0, -beta * p_lo, p_lo * np.expm1(-beta * dl) / safe)
    rho = np.einsum('nik,nk,njk->nij', U, p, U.conj())
    M = np.einsum('nki,nkl,nlj->nij', U.conj(), Xbar, U)
    out = np.einsum('nik,nkl,njl->nij', U, G * M, U.conj())
    rx = np.real(np.einsum('nij,nij->n', rho.conj(), Xbar))
    return herm(out + beta * rx[:, None, None] * rho)


def dual_vjp(R: Relaxation, nu, beta: float, qbar, gbar=None, params=None):
    """Cotangents (qbar per instance, gbar per message) of (Q_beta(nu), grad Q_beta(nu)) ->
    (nu_bar, param_bar).  With B the linear map messages -> augmented Hamiltonians
    (B nu)_e = -sum_children 1 (x) nu + sum_parents nu, grad Q_beta = B^* rho (chain rule of
    the Lipschitz lemma), so with Y_e = qbar rho_e + D rho_e[(B gbar)_e]:
    nu_bar = B^* Y (Y_f - Tr_{e\\f} Y_e) and param_bar_p = sum_t <Y_e(t), dh_t/dc_p>.
    beta = 0: Q itself, Y_e = qbar mu_e (ground projector), gbar must be None."""
    h = None if params is None else h_at_params(R, params)
    th = R.thetas(nu, h=h)
    if gbar is not None:
        X = R.thetas(gbar, with_h=False)
    Y = {}
    for D, ids in R.cgroups.items():
        qb = np.asarray(qbar, dtype=np.float64)[R.inst[ids]]
        if beta > 0:
            lam, U = np.linalg.eigh(th[D])
            w = np.exp(-beta * (lam - lam[:, :1]))
            p = w / w.sum(axis=1, keepdims=True)
            rho = herm(np.einsum('nik,nk,njk->nij', U, p, U.conj()))
            Yd = qb[:, None, None] * rho
            if gbar is not None:
                Yd = Yd + gibbs_vjp_batch(th[D], beta, X[D])
        else:
            if gbar is not None:
                raise ValueError("the subgradient has no derivative: gbar must be None at beta = 0")
            lam, U = np.linalg.eigh(th[D])
            tau = 1e-9 * np.maximum(1.0, np.linalg.norm(th[D], axis=(1, 2)))
            sel = (lam <= lam[:, :1] + tau[:, None]).astype(np.float64)
            mu = herm(np.einsum('nik,nk,njk->nij', U, sel / sel.sum(axis=1, keepdims=True), U.conj()))
            Yd = qb[:, None, None] * mu
        Y[D] = Yd
    nu_bar = R._grad_from_marginals(Y)
    npar = 0 if R.desc.params is None else len(R.desc.params)
    pbar = np.zeros(npar)
    for e, p, B in term_params(R):
        D = int(R.D[e])
        pbar[p] += float(np.real(np.vdot(Y[D][R.cslot[e]], B)))
    return nu_bar, pbar


def unrolled_bound(R: Relaxation, beta: float, T: int, params=None, nu0=None, L=None):
    """B_T = Q(nu^T) per instance, nu^T = T steps of Algorithm 2 at fixed beta from nu0
    (zeta0 = nu0, theta0 = 1), everything at parameters `params`."""
    h = None if params is None else h_at_params(R, params)
    L = R.lipschitz(beta) if L is None else L
    nu = R.zeros() if nu0 is None else R.copy(nu0)
    ze = R.copy(nu)
    th = 1.0
    for _ in range(T):
        eta = R.axpby(1.0 - th, nu, th, ze)
        g = _grad_beta_h(R, eta, beta, h)
        ze = R.symmetrise({k: ze[k] + g[k] / (th * L) for k in ze})
        nu = R.symmetrise(R.axpby(1.0 - th, nu, th, ze))
        th = theta_next(th)
    lm = {D: np.linalg.eigvalsh(t)[:, 0] for D, t in R.thetas(nu, h=h).items()}
    return R._per_instance(lm), nu


def _grad_beta_h(R, eta, beta, h):
    th = R.thetas(eta, h=h)
    rho = {}
    for D, t in th.items():
        lam, U = np.linalg.eigh(t)
        w = np.exp(-beta * (lam - lam[:, :1]))
        p = w / w.sum(axis=1, keepdims=True)
        rho[D] = herm(np.einsum('nik,nk,njk->nij', U, p, U.conj()))
    return R._grad_from_marginals(rho)


def unrolled_bound_grad(R: Relaxation, beta: float, T: int, params=None, nu0=None, qbar=None, L=None):
    """Reverse mode through `unrolled_bound`: returns (B_T, d<qbar, B_T>/d params, d/d nu0).

    Backward of one step (eta = (1-th) nu + th ze; g = grad Q_beta(eta); ze' = ze + g/(th L);
    nu' = (1-th) nu + th ze') with cotangents (a, b) of (nu', ze'):
        b_tot = b + th a;  g_bar = b_tot / (th L);  (eta_bar, c_bar) = VJP of g at eta;
        a <- (1-th)(a + eta_bar);  b <- b_tot + th eta_bar.
    At the start of the stage zeta0 = nu0, so nu0_bar = a + b."""
    L = R.lipschitz(beta) if L is None else L
    h = None if params is None else h_at_params(R, params)
    qbar = np.ones(R.n_inst) if qbar is None else np.asarray(qbar, dtype=np.float64)
    nu = R.zeros() if nu0 is None else R.copy(nu0)
    ze = R.copy(nu)
    th = 1.0
    etas, ths = [], []
    for _ in range(T):
        eta = R.axpby(1.0 - th, nu, th, ze)
        etas.append(eta)
        ths.append(th)
        g = _grad_beta_h(R, eta, beta, h)
        ze = R.symmetrise({k: ze[k] + g[k] / (th * L) for k in ze})
        nu = R.symmetrise(R.axpby(1.0 - th, nu, th, ze))
        th = theta_next(th)
    lm = {D: np.linalg.eigvalsh(t)[:, 0] for D, t in R.thetas(nu, h=h).items()}
    bound = R._per_instance(lm)
    a, cbar = dual_vjp(R, nu, 0.0, qbar, None, params)
    b = R.zeros()
    zero_q = np.zeros(R.n_inst)
    for k in range(T - 1, -1, -1):
        th = ths[k]
        btot = R.axpby(1.0, b, th, a)
        gbar = {D: v / (th * L) for D, v in btot.items()}
        etabar, cb = dual_vjp(R, etas[k], beta, zero_q, gbar, params)
        cbar = cbar + cb
        a = {D: (1.0 - th) * (a[D] + etabar[D]) for D in a}
        b = R.axpby(1.0, btot, th, etabar)
    nu0bar = R.axpby(1.0, a, 1.0, b)
    return bound, cbar, nu0bar
