"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each checks a closed form, an
invariant, a brute-force computation or an exact special case (see each docstring
for the passage it follows).
"""
import itertools
import math

import numpy as np
import pytest

import lrh_workloads as W
from oracle import exact as E
from oracle import lrh_oracle as O

from conftest import golden, read_reference_energies


# ------------------------------------------------------------------------------------------
# brute-force lift / partial trace from the index definition (not the oracle's einsum)
# ------------------------------------------------------------------------------------------

def bf_index(digits, dims):
    i = 0
    for dgt, d in zip(digits, dims):
        i = i * d + dgt
    return i


def bf_lift(X, dims_e, pos):
    """(1_{e\\f} (x) X)[i, j] = X[a(i), a(j)] * delta(rest(i), rest(j)) with site order of e."""
    De = int(np.prod(dims_e))
    out = np.zeros((De, De), dtype=np.complex128)
    fd = [dims_e[p] for p in pos]
    for di in itertools.product(*[range(d) for d in dims_e]):
        for dj in itertools.product(*[range(d) for d in dims_e]):
            if any(di[k] != dj[k] for k in range(len(dims_e)) if k not in pos):
                continue
            a = bf_index([di[p] for p in pos], fd)
            b = bf_index([dj[p] for p in pos], fd)
            out[bf_index(di, dims_e), bf_index(dj, dims_e)] = X[a, b]
    return out


def bf_ptrace(A, dims_e, pos):
    fd = [dims_e[p] for p in pos]
    rest = [k for k in range(len(dims_e)) if k not in pos]
    Df = int(np.prod(fd))
    out = np.zeros((Df, Df), dtype=np.complex128)
    for da in itertools.product(*[range(d) for d in fd]):
        for db in itertools.product(*[range(d) for d in fd]):
            s = 0
            for dr in itertools.product(*[range(dims_e[k]) for k in rest]):
                di = [0] * len(dims_e)
                dj = [0] * len(dims_e)
                for p, x, y in zip(pos, da, db):
                    di[p], dj[p] = x, y
                for k, x in zip(rest, dr):
                    di[k] = dj[k] = x
                s += A[bf_index(di, dims_e), bf_index(dj, dims_e)]
            out[bf_index(da, fd), bf_index(db, fd)] = s
    return out


@pytest.mark.parametrize("dims_e,pos", [((2, 2), (0,)), ((2, 2), (1,)), ((2, 2, 2), (0, 2)),
                                        ((2, 3, 2), (1,)), ((3, 2, 2), (0, 2)),
                                        ((2, 2, 2, 2), (1, 2))])
def test_lift_and_partial_trace_brute_force(dims_e, pos):
    rng = np.random.default_rng(7)
    De = int(np.prod(dims_e))
    Df = int(np.prod([dims_e[p] for p in pos]))
    X = rng.normal(size=(Df, Df)) + 1j * rng.normal(size=(Df, Df))
    A = rng.normal(size=(De, De)) + 1j * rng.normal(size=(De, De))
    np.testing.assert_allclose(O.lift(X, dims_e, pos), bf_lift(X, dims_e, pos), atol=1e-14)
    np.testing.assert_allclose(O.ptrace(A, dims_e, pos), bf_ptrace(A, dims_e, pos), atol=1e-13)
    # adjointness <Tr_{e\f} A, X> = <A, 1 (x) X>, the identity behind the Lagrangian rewrite
    lhs = np.vdot(O.ptrace(A, dims_e, pos), X)
    rhs = np.vdot(A, O.lift(X, dims_e, pos))
    assert abs(lhs - rhs) < 1e-12


def test_basis_convention_is_kron():
    """A on the first (lower-numbered) site, B on the second == np.kron(A, B)."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=(2, 2))
    B = rng.normal(size=(3, 3))
    full = O.lift(A, (2, 3), (0,)) @ O.lift(B, (2, 3), (1,))
    np.testing.assert_allclose(full, np.kron(A, B), atol=1e-15)


# ------------------------------------------------------------------------------------------
# poset
# ------------------------------------------------------------------------------------------

def test_poset_matches_figure_1():
    """Fig. 1: chain of 5 sites with Y_3 -> exactly the drawn covering arrows."""
    arrows = set()
    with open(golden("fig1_poset.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p, c = [x.strip() for x in line.split("->")]
            arrows.add((tuple(int(ch) - 1 for ch in p), tuple(int(ch) - 1 for ch in c)))
    d = W.random_chain(5, seed=0, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    got = {(R.clusters[e], R.clusters[f]) for (e, f) in R.msgs}
    assert got == arrows
    assert len(R.clusters) == 12


def test_poset_plaquette_children_are_its_four_bonds():
    """Covering relation, not 'one site fewer': a plaquette's children are its 4 edges."""
    d = W.tfim_plaquette_batch([3], [1.0])
    R = O.Relaxation(d)
    for e, c in enumerate(R.clusters):
        if len(c) == 4:
            ch = [R.clusters[f] for f in R.children[e]]
            assert len(ch) == 4 and all(len(x) == 2 for x in ch)
        if len(c) == 2:
            assert len(R.parents[e]) == 2 and len(R.children[e]) == 2
        if len(c) == 1:
            assert len(R.parents[e]) == 4


# ------------------------------------------------------------------------------------------
# dual value: closed forms, weak duality, gauge, exact special cases
# ------------------------------------------------------------------------------------------

def test_anderson_bound_tfim_chain():
    """Q(0) is the Anderson bound (Sec. 3.1): 15 * (-1) + 16 * (-0.5) = -23."""
    ref = read_reference_energies()
    R = O.Relaxation(W.workload_c1())
    assert R.Q(R.zeros())[0] == pytest.approx(ref["tfim_chain_n16_anderson"], abs=1e-12)


def test_anderson_bound_equals_sum_of_term_minima():
    d = W.random_chain(6, seed=11)
    R = O.Relaxation(d)
    want = math.fsum(np.linalg.eigvalsh(m)[0] for _, m in d.terms())
    assert R.Q(R.zeros())[0] == pytest.approx(want, abs=1e-12)


def test_heisenberg_square_level1_closed_form():
    """Singlets on every bond are locally consistent: f_1* = -3 J per bond, and the Gibbs
    gradient vanishes at nu = 0 by SU(2) symmetry, so zero messages are optimal."""
    d = W.workload_c2(32)
    R = O.Relaxation(d)
    assert R.Q(R.zeros())[0] == pytest.approx(-6144.0, abs=1e-9)
    small = O.Relaxation(W.heisenberg_square(4))
    for beta in (1.0, 64.0, 1024.0):
        _, g = small.grad_beta(small.zeros(), beta)
        assert max(np.abs(v).max() for v in g.values()) < 1e-12


def test_frustration_free_ferromagnet_is_exact():
    """Frustration-free H: every level equals E0 = Anderson (Sec. 3.1.1)."""
    d = W.heisenberg_chain(6, J=-1.0)
    R = O.Relaxation(d)
    E0 = E.ground_energy(d)
    assert E0 == pytest.approx(-5.0, abs=1e-10)
    assert R.Q(R.zeros())[0] == pytest.approx(E0, abs=1e-12)


@pytest.mark.parametrize("maker", [
    lambda: W.tfim_chain(8, 1.0, 1.0),
    lambda: W.random_chain(7, seed=3),
    lambda: W.random_chain(7, seed=4, top_len=3, subintervals=True),
    lambda: W.heisenberg_graph(8, W.square_edges(2, periodic=False, offset=0)
                               + [(4, 5), (5, 6), (6, 7), (3, 4)], name="h8"),
    lambda: W.xxz_triangular(3, 0.5, seed=2),
    lambda: W.random_chain(7, seed=4, top_len=3, two_level=True),
    lambda: _grid6_plaquettes_two_level(),
])
def test_weak_duality_random_messages(maker):
    """Any nu gives a lower bound: Q(nu) <= E0 (partial Lagrangian, Sec. 4.1)."""
    d = maker()
    R = O.Relaxation(d)
    E0 = E.ground_energy(d)
    for seed in range(4):
        nu = R.draw(seed, scale=0.7)
        assert R.Q(nu)[0] <= E0 + 1e-10


def test_gauge_invariance():
    """nu_{e->f} += c 1 lowers theta_e by c 1 and raises theta_f by c 1 (both are traces of
    identities), so Q is unchanged: the trace of a message is a gauge."""
    d = W.random_chain(6, seed=5, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    nu = R.draw(1, 0.5)
    q0 = R.Q(nu)[0]
    for m in [0, 3, R.n_msgs - 1]:
        nu2 = R.copy(nu)
        Df = int(R.mDf[m])
        R.set(nu2, m, R.get(nu2, m) + 0.37 * np.eye(Df))
        assert R.Q(nu2)[0] == pytest.approx(q0, abs=1e-12)


def _exact_messages_whole_cluster(R, desc):
    """Messages that move every term onto the single top cluster (whole system).

    Site term h_v is sent to one edge containing v (nu_{e->v} = -h_v), every edge term
    plus what it received is sent to the top (nu_{top->e} = -(h_e + sum lift h_v)).  Then
    theta_v = theta_e = 0 and theta_top = H, so Q(nu) must equal E0 exactly."""
    nu = R.zeros()
    top = max(range(R.n_clusters), key=lambda e: len(R.clusters[e]))
    ctop = R.clusters[top]
    sd = R.site_dim
    received = {}
    for v in range(desc.n_sites):
        ev = R.index[(v,)]
        if ev not in R.h:
            continue
        e = R.parents[ev][0]
        ce = R.clusters[e]
        R.set(nu, R.msg_index[(e, ev)], -R.h[ev])
        pos = (ce.index(v),)
        received[e] = received.get(e, 0) + bf_lift(R.h[ev], [sd[s] for s in ce], pos)
    for e in R.children[top]:
        ce = R.clusters[e]
        tot = R.h.get(e, 0) + received.get(e, 0)
        R.set(nu, R.msg_index[(top, e)], -np.asarray(tot) if not np.isscalar(tot) else
              np.zeros((R.D[e], R.D[e])))
    return nu


@pytest.mark.parametrize("maker", [lambda: W.tfim_chain(6, 1.0, 0.7),
                                   lambda: W.random_chain(5, seed=9)])
def test_whole_system_cluster_attains_E0(maker):
    """One cluster holding every site: the relaxation is exact (Sec. 3.2: E0 = f*_{C+m}),
    and an explicit message assignment reaches Q = lambda_min(H) = E0."""
    d = W.whole_system(maker())
    R = O.Relaxation(d)
    nu = _exact_messages_whole_cluster(R, d)
    assert R.Q(nu)[0] == pytest.approx(E.ground_energy(d), abs=1e-11)


# ------------------------------------------------------------------------------------------
# smoothing, gradients, subgradients
# ------------------------------------------------------------------------------------------

def test_smoothing_sandwich():
    """Q_beta <= Q <= Q_beta + Gamma_G / beta (smoothing-error lemma)."""
    d = W.random_chain(6, seed=2, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    for beta in (0.5, 3.0, 40.0):
        nu = R.draw(3, 0.5)
        q, qb = R.Q(nu)[0], R.Q_beta(nu, beta)[0]
        assert qb <= q + 1e-12
        assert q <= qb + R.Gamma / beta + 1e-12


def _inner(R, a, b):
    return math.fsum(float(np.real(np.vdot(a[k], b[k]))) for k in a)


@pytest.mark.parametrize("maker", [lambda: W.random_chain(5, seed=1),
                                   lambda: W.random_chain(5, seed=8, top_len=3, subintervals=True),
                                   lambda: W.xxz_triangular(3, 0.5, seed=1),
                                   lambda: W.random_chain(6, seed=8, top_len=3, two_level=True),
                                   lambda: _grid6_plaquettes_two_level()])
def test_smoothed_gradient_matches_finite_differences(maker):
    """grad_{nu_{e->f}} Q_beta = rho_f - Tr_{e\\f} rho_e (Sec. 4.1.2 / 4.2.2)."""
    d = maker()
    R = O.Relaxation(d)
    beta = 2.5
    nu = R.draw(4, 0.4)
    X = R.draw(5, 1.0)
    _, g = R.grad_beta(nu, beta)
    t = 1e-5
    qp = R.Q_beta(R.axpby(1, nu, t, X), beta)[0]
    qm = R.Q_beta(R.axpby(1, nu, -t, X), beta)[0]
    fd = (qp - qm) / (2 * t)
    assert fd == pytest.approx(_inner(R, g, X), rel=1e-6, abs=1e-7)


def test_subgradient_is_a_supergradient():
    """Q is concave and mu_f - Tr mu_e lies in its superdifferential (Sec. 4.1.1):
    Q(nu') <= Q(nu) + <g(nu), nu' - nu> for all nu'."""
    d = W.random_chain(6, seed=6, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    nu = R.draw(10, 0.5)
    q, g = R.subgrad(nu)
    for s in range(6):
        nu2 = R.draw(20 + s, 0.5)
        diff = R.axpby(1, nu2, -1, nu)
        assert R.Q(nu2)[0] <= q[0] + _inner(R, g, diff) + 1e-10


def test_gibbs_lipschitz():
    """||rho(K) - rho(K')||_F <= (beta/2) ||K - K'||_F (Lipschitz lemma, m_F = 2)."""
    rng = np.random.default_rng(3)
    for D in (2, 4, 8):
        for beta in (0.3, 2.0, 10.0):
            K = W.gue(rng, D)
            K2 = K + 0.3 * W.gue(rng, D)
            r1 = _gibbs(K, beta)
            r2 = _gibbs(K2, beta)
            assert np.linalg.norm(r1 - r2) <= beta / 2 * np.linalg.norm(K - K2) + 1e-12


def _gibbs(K, beta):
    """Gibbs state via the exponential series on a shifted spectrum (independent of eigh use
    in the oracle): rho = e^{-beta K}/Tr e^{-beta K}."""
    from scipy.linalg import expm
    M = expm(-beta * (K - np.eye(len(K)) * np.linalg.eigvalsh(K)[0]))
    return M / np.trace(M)


def test_gibbs_state_matches_matrix_exponential():
    d = W.random_chain(4, seed=12)
    R = O.Relaxation(d)
    nu = R.draw(2, 0.3)
    F, rho = R.gibbs(nu, 3.0)
    th = R.thetas(nu)
    for D in th:
        for j in range(len(th[D])):
            np.testing.assert_allclose(rho[D][j], _gibbs(th[D][j], 3.0), atol=1e-12)
            lam = np.linalg.eigvalsh(th[D][j])
            from scipy.special import logsumexp
            assert F[D][j] == pytest.approx(-logsumexp(-3.0 * lam) / 3.0, abs=1e-12)


def test_smoothed_dual_gradient_lipschitz_two_local():
    """||grad Q_b(nu) - grad Q_b(nu')|| <= beta (Delta_G + d)/2 ||nu - nu'|| on traceless nu."""
    d = W.random_chain(6, seed=13)
    R = O.Relaxation(d)
    beta = 1.5
    L = R.lipschitz(beta)
    assert R.Lambda == R.Delta_G() + 2

    def traceless(nu):
        return {k: v - np.trace(v, axis1=1, axis2=2)[:, None, None] / k * np.eye(k) for k, v in nu.items()}
    for s in range(4):
        a = traceless(R.draw(30 + s, 0.8))
        b = traceless(R.draw(40 + s, 0.8))
        _, ga = R.grad_beta(a, beta)
        _, gb = R.grad_beta(b, beta)
        lhs = math.sqrt(_inner(R, R.axpby(1, ga, -1, gb), R.axpby(1, ga, -1, gb)))
        rhs = L * math.sqrt(_inner(R, R.axpby(1, a, -1, b), R.axpby(1, a, -1, b)))
        assert lhs <= rhs + 1e-12


def test_gibbs_vjp_matches_finite_differences():
    """Daleckii-Krein VJP of rho_beta (textbook matrix calculus) vs central differences,
    including an exactly degenerate spectrum."""
    rng = np.random.default_rng(5)
    cases = [W.gue(rng, 4), W.gue(rng, 8), np.kron(W.X, W.X) + np.kron(W.Y, W.Y) + np.kron(W.Z, W.Z)]
    for K in cases:
        D = len(K)
        rb = W.gue(rng, D)
        Edir = W.gue(rng, D)
        beta = 1.7
        tb = O.gibbs_vjp(K, beta, rb)
        h = 1e-6
        fp = np.real(np.vdot(rb, _gibbs(K + h * Edir, beta)))
        fm = np.real(np.vdot(rb, _gibbs(K - h * Edir, beta)))
        assert (fp - fm) / (2 * h) == pytest.approx(np.real(np.vdot(tb, Edir)), rel=1e-6, abs=1e-8)


# ------------------------------------------------------------------------------------------
# the two algorithms
# ------------------------------------------------------------------------------------------

def test_theta_sequence_identity():
    """theta_{k+1} = (sqrt(th^4 + 4 th^2) - th^2)/2 solves (1 - t')/t'^2 = 1/t^2 (Tseng)."""
    th = 1.0
    for _ in range(200):
        tn = O.theta_next(th)
        assert (1 - tn) / tn ** 2 == pytest.approx(1 / th ** 2, rel=1e-12)
        assert 0 < tn < th
        th = tn


def test_messages_stay_traceless():
    """Every gradient/subgradient has trace 1 - 1 = 0, so nu stays traceless."""
    d = W.random_chain(6, seed=14, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    nu = O.nesterov(R, [(2.0, 40), (4.0, 40)])
    for v in nu.values():
        assert np.abs(np.trace(v, axis1=1, axis2=2)).max() < 1e-12
    nb, _, nT, _ = O.subgradient(R, 60)
    for v in nT.values():
        assert np.abs(np.trace(v, axis1=1, axis2=2)).max() < 1e-12


def test_time_reversal_keeps_site_messages_zero():
    """Zero-field XXZ is time-reversal invariant; spin-1/2 site marginals of TR-invariant
    states are 1/2, so every message into a single site stays zero."""
    d = W.xxz_triangular(3, 0.5, seed=3)
    R = O.Relaxation(d)
    nu = O.nesterov(R, [(4.0, 30)])
    assert np.abs(nu[2]).max() < 1e-12
    assert np.abs(nu[4]).max() > 1e-3


def test_subgradient_c1_bracket():
    """C1: Anderson <= q_best <= E0 (weak duality), q_best nondecreasing along the run."""
    ref = read_reference_energies()
    d = W.workload_c1()
    R = O.Relaxation(d)
    nb, qb, _, hist = O.subgradient(R, 400)
    assert ref["tfim_chain_n16_anderson"] <= qb[0] <= ref["tfim_chain_n16_E0"]
    assert qb[0] == pytest.approx(hist.max(), abs=0)
    assert R.Q(nb)[0] == pytest.approx(qb[0], abs=1e-12)
    assert qb[0] > -17.3   # substantial progress from -23 within 400 steps


def test_free_fermion_energy_matches_lanczos_and_fixture():
    ref = read_reference_energies()
    assert E.tfim_open_chain_E0(16, 1.0, 0.5) == pytest.approx(ref["tfim_chain_n16_E0"], abs=1e-12)
    for n, J, h in [(6, 1.0, 0.5), (8, 0.7, 1.3)]:
        assert E.tfim_open_chain_E0(n, J, h) == pytest.approx(
            E.ground_energy(W.tfim_chain(n, J, h)), abs=1e-10)


@pytest.mark.parametrize("seed,rotate", [(1, False), (2, False), (3, True), (4, True)])
def test_level1_exact_on_commuting_trees(seed, rotate):
    """Diagonal Hamiltonians on trees (Sec. 3.1.1) and commuting ones (Thm. 2): level 1 is
    exact; the smoothed solver's certified value reaches the brute-force minimum."""
    d = W.classical_ising_tree(8, seed, rotate=rotate)
    R = O.Relaxation(d)
    E0 = E.classical_min(W.classical_ising_tree(8, seed, rotate=False))
    nu = O.nesterov(R, O.doubling_schedule(1.0, 4096.0, 1300))
    q, margin = R.certify(nu)
    assert q[0] - margin[0] <= E0 + 1e-12
    assert q[0] == pytest.approx(E0, abs=1e-6)


def test_monogamy_three_site_heisenberg():
    """Sec. 2 monogamy example: level 1 gives -6 (singlets on both edges), E0 = -4."""
    ref = read_reference_energies()
    d = W.heisenberg_chain(3)
    R = O.Relaxation(d)
    assert E.ground_energy(d) == pytest.approx(ref["heisenberg_chain3_E0"], abs=1e-12)
    nu = O.nesterov(R, [(8.0, 50)])
    assert R.Q(nu)[0] == pytest.approx(ref["heisenberg_chain3_level1"], abs=1e-10)


def test_tseng_rate_bound():
    """Alg. 2 at fixed beta: Q_b* - Q_b(nu_T) <= 2 L R^2 / (T+1)^2 (Tseng, Cor. 1)."""
    d = W.random_chain(5, seed=21)
    R = O.Relaxation(d)
    beta = 4.0
    L = R.lipschitz(beta)
    ref = O.nesterov(R, [(beta, 3000)])
    qstar = R.Q_beta(ref, beta)[0]
    Rn = math.sqrt(_inner(R, ref, ref))
    for T in (5, 20, 80):
        nu = O.nesterov(R, [(beta, T)])
        gap = qstar - R.Q_beta(nu, beta)[0]
        assert gap <= 2 * L * Rn ** 2 / (T + 1) ** 2 + 1e-9


def test_interval_hierarchy_monotone_and_exact_at_full_length():
    """E0 = f*_n >= ... >= f*_t (Sec. 3.2) and (E0 - f*_t)/n <= 1/t when 2||h|| <= 1."""
    n = 5
    base = W.random_chain(n, seed=31, scale=1.0)
    # rescale every term to 2||h|| <= 1
    terms = [(s, m / (2 * np.max(np.abs(np.linalg.eigvalsh(m))))) for s, m in base.terms()]
    b = W._Builder("scaled", n)
    for s, m in terms:
        b.add_term(s, m)
    E0 = None
    vals = []
    for t in range(2, n + 1):
        b.tops = [tuple(range(i, i + t)) for i in range(n - t + 1)]
        d = b.build(real=False, subintervals=True)
        if E0 is None:
            E0 = E.ground_energy(d)
        R = O.Relaxation(d)
        nu = O.nesterov(R, O.doubling_schedule(1.0, 2048.0, 1200))
        q, mg = R.certify(nu)
        vals.append(q[0] - mg[0])
        assert (E0 - vals[-1]) / n <= 1.0 / t + 1e-9
        assert vals[-1] <= E0 + 1e-12
    for a, c in zip(vals, vals[1:]):
        assert c >= a - 2e-3
    assert vals[-1] == pytest.approx(E0, abs=5e-3)


# ------------------------------------------------------------------------------------------
# reverse mode (gradient of the certified bound with respect to couplings)
# ------------------------------------------------------------------------------------------

def test_unrolled_bound_gradient_zero_steps_is_hellmann_feynman():
    """T = 0: B_0 = Anderson bound = sum_e J_e lambda_min(XX+YY+Delta ZZ); each bond's
    derivative is lambda_min(XX+YY+Delta ZZ) = -(2 + Delta)."""
    d = W.xxz_triangular(3, 0.5, seed=5)
    R = O.Relaxation(d)
    B, cb, _ = O.unrolled_bound_grad(R, 4.0, 0)
    np.testing.assert_allclose(cb, -2.5, atol=1e-12)
    assert B[0] == pytest.approx(-2.5 * d.params.sum(), abs=1e-10)


@pytest.mark.parametrize("T,two", [(3, False), (8, False), (3, True)])
def test_unrolled_bound_gradient_matches_central_differences(T, two):
    d = W.xxz_triangular(3, 0.5, seed=5, n_bonds=5, two_level=two)
    R = O.Relaxation(d)
    _, cb, _ = O.unrolled_bound_grad(R, 4.0, T)
    c0 = d.params.copy()
    h = 1e-6
    for p in d.meta["bonds"]:
        cp, cm = c0.copy(), c0.copy()
        cp[p] += h
        cm[p] -= h
        fd = (O.unrolled_bound(R, 4.0, T, cp)[0][0] - O.unrolled_bound(R, 4.0, T, cm)[0][0]) / (2 * h)
        assert cb[p] == pytest.approx(fd, abs=1e-7)


def test_unrolled_bound_gradient_wrt_initial_messages():
    d = W.random_chain(5, seed=3)
    R = O.Relaxation(d)
    nu0 = R.draw(1, 0.3)
    _, _, n0b = O.unrolled_bound_grad(R, 2.0, 5, nu0=nu0)
    X = R.draw(2, 1.0)
    t = 1e-6
    fp = O.unrolled_bound(R, 2.0, 5, nu0=R.axpby(1, nu0, t, X))[0][0]
    fm = O.unrolled_bound(R, 2.0, 5, nu0=R.axpby(1, nu0, -t, X))[0][0]
    assert (fp - fm) / (2 * t) == pytest.approx(_inner(R, n0b, X), abs=1e-7)


def test_dual_vjp_is_the_transposed_hessian():
    """<gbar, d grad Q_beta[X]> = <VJP(gbar), X> and the qbar part is qbar * grad."""
    d = W.random_chain(5, seed=7, top_len=3, subintervals=True)
    R = O.Relaxation(d)
    beta = 1.3
    nu = R.draw(3, 0.4)
    gbar = R.draw(4, 1.0)
    X = R.draw(5, 1.0)
    vb, _ = O.dual_vjp(R, nu, beta, np.zeros(1), gbar)
    t = 1e-6
    _, gp = R.grad_beta(R.axpby(1, nu, t, X), beta)
    _, gm = R.grad_beta(R.axpby(1, nu, -t, X), beta)
    fd = (_inner(R, gbar, gp) - _inner(R, gbar, gm)) / (2 * t)
    assert fd == pytest.approx(_inner(R, vb, X), abs=1e-7)
    vq, _ = O.dual_vjp(R, nu, beta, np.array([2.5]), None)
    _, g = R.grad_beta(nu, beta)
    for k in g:
        np.testing.assert_allclose(vq[k], 2.5 * g[k], atol=1e-13)


def test_batched_gibbs_vjp_equals_single():
    rng = np.random.default_rng(9)
    K = np.stack([W.gue(rng, 8) for _ in range(5)] + [np.kron(np.kron(W.X, W.X) + np.kron(W.Y, W.Y), np.eye(2))])
    X = np.stack([W.gue(rng, 8) for _ in range(6)])
    got = O.gibbs_vjp_batch(K, 2.3, X)
    for j in range(len(K)):
        np.testing.assert_allclose(got[j], O.gibbs_vjp(K[j], 2.3, X[j]), atol=1e-12)


# ------------------------------------------------------------------------------------------
# two-level family: top clusters and their maximal pairwise overlaps only, every term split
# evenly over the top clusters holding its support
# ------------------------------------------------------------------------------------------

def _grid6_plaquettes_two_level():
    """Open 2 x 3 Heisenberg grid (sites x + 3y) with a field, tops = its two 2 x 2 plaquettes."""
    edges = [(0, 1), (1, 2), (3, 4), (4, 5), (0, 3), (1, 4), (2, 5)]
    d = W.heisenberg_graph(6, edges, field_x=0.3, name="grid6")
    return W.with_tops(d, [(0, 1, 3, 4), (1, 2, 4, 5)], two_level=True)


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(2 ** n, 2 ** n)) + 1j * rng.normal(size=(2 ** n, 2 ** n))
    rho = G @ G.conj().T
    return rho / np.trace(rho).real


def test_two_level_family_on_a_chain_is_windows_and_overlaps():
    """Windows of length t on an open chain of n sites: the maximal pairwise intersections are
    the n - t overlaps of consecutive windows; each inner window covers two of them, each
    overlap has the two windows around it as parents (Hasse diagram of the inclusion order)."""
    n, t = 9, 4
    R = O.Relaxation(W.random_chain(n, seed=2, top_len=t, two_level=True))
    windows = [tuple(range(i, i + t)) for i in range(n - t + 1)]
    overlaps = [tuple(range(i + 1, i + t)) for i in range(n - t)]
    assert sorted(R.clusters) == sorted(windows + overlaps)
    for i, w in enumerate(windows):
        e = R.index[w]
        want = [o for o in overlaps if set(o) <= set(w)]
        assert sorted(R.clusters[f] for f in R.children[e]) == want
        assert len(want) == (1 if i in (0, n - t) else 2)
        assert R.parents[e] == []
    for i, o in enumerate(overlaps):
        f = R.index[o]
        assert sorted(R.clusters[e] for e in R.parents[f]) == [windows[i], windows[i + 1]]
        assert R.children[f] == [] and f not in R.h
    # the grid: its two plaquettes overlap in the middle bond only
    G = O.Relaxation(_grid6_plaquettes_two_level())
    assert sorted(G.clusters) == sorted([(1, 4), (0, 1, 3, 4), (1, 2, 4, 5)])


@pytest.mark.parametrize("maker,n", [
    (lambda: W.random_chain(6, seed=12, top_len=3, two_level=True), 6),
    (lambda: W.interval_chain_gue(6, 4, eps=0.3, seed=2, two_level=True), 6),
    (_grid6_plaquettes_two_level, 6),
])
def test_two_level_terms_keep_the_energy_of_any_state(maker, n):
    """The split terms lose nothing: for a random global state rho, sum over clusters of
    Tr(h_e Tr_rest rho) equals Tr(H rho) with H built densely from the terms."""
    d = maker()
    R = O.Relaxation(d)
    H = E.dense_H(d)
    for seed in range(2):
        rho = _random_state(n, seed)
        tot = 0.0
        for e, h in R.h.items():
            pos = R.clusters[e]
            tot += np.trace(h @ bf_ptrace(rho, [2] * n, pos)).real
        assert tot == pytest.approx(np.trace(H @ rho).real, abs=1e-12)


@pytest.mark.parametrize("maker,n", [
    (lambda: W.random_chain(6, seed=13, top_len=3, two_level=True), 6),
    (_grid6_plaquettes_two_level, 6),
])
def test_two_level_lagrangian_is_message_free_on_consistent_marginals(maker, n):
    """Marginals of one global state satisfy every covering constraint, so the message terms of
    the partial Lagrangian (Sec. 4.1, Sec. 4.2) cancel: sum_e Tr(theta_e(nu) mu_e) = Tr(H rho)
    for every nu."""
    d = maker()
    R = O.Relaxation(d)
    H = E.dense_H(d)
    rho = _random_state(n, 7)
    mu = {e: bf_ptrace(rho, [2] * n, R.clusters[e]) for e in range(R.n_clusters)}
    for seed in range(3):
        nu = R.draw(seed, 0.8)
        tot = sum(np.trace(R.theta(nu, e) @ mu[e]).real for e in range(R.n_clusters))
        assert tot == pytest.approx(np.trace(H @ rho).real, abs=1e-11)


def test_two_level_single_window_is_exact():
    """One window over the whole chain: no overlaps, theta = H, so Q(0) = E0 (Sec. 3.2)."""
    d = W.random_chain(6, seed=14, top_len=6, two_level=True)
    R = O.Relaxation(d)
    assert R.n_clusters == 1
    assert R.Q(R.zeros())[0] == pytest.approx(E.ground_energy(d), abs=1e-11)


@pytest.mark.parametrize("seed,rotate", [(1, False), (3, True)])
def test_two_level_exact_on_commuting_trees(seed, rotate):
    """Edges of a tree as tops, inner sites as overlaps (leaf sites are no clusters): commuting
    terms on a tree are still solved exactly, as by the full level-1 family."""
    d0 = W.classical_ising_tree(8, seed, rotate=rotate)
    d = W.with_tops(d0, list(d0.tops()), two_level=True)
    R = O.Relaxation(d)
    assert all(len(c) == 2 or len(R.parents[e]) >= 2 for e, c in enumerate(R.clusters))
    E0 = E.classical_min(W.classical_ising_tree(8, seed, rotate=False))
    nu = O.nesterov(R, O.doubling_schedule(1.0, 4096.0, 1300))
    q, margin = R.certify(nu)
    assert q[0] - margin[0] <= E0 + 1e-12
    assert q[0] == pytest.approx(E0, abs=1e-6)


def test_two_level_optimum_equals_the_interval_hierarchy():
    """On a chain, consistency of consecutive windows on their overlaps implies consistency on
    every shorter interval, and each split term is evaluated on marginals the windows share,
    so windows + overlaps have the optimum of Y_t (Sec. 3.2).  Both optima are approached with
    Algorithm 2 and certified; they agree to the accuracy the runs reach."""
    n, t = 5, 3
    base = W.random_chain(n, seed=33)
    vals = {}
    for two in (False, True):
        d = W.with_tops(base, [tuple(range(i, i + t)) for i in range(n - t + 1)],
                        subintervals=not two, two_level=two)
        R = O.Relaxation(d)
        nu = O.nesterov(R, O.doubling_schedule(1.0, 16384.0, 6000))
        q, mg = R.certify(nu)
        vals[two] = q[0] - mg[0]
        assert vals[two] <= E.ground_energy(d) + 1e-12
    # both runs still sit 1e-4 .. 1e-3 below the common optimum (their difference falls
    # from 1.5e-3 at 3000 iterations to 5e-5 at 12000)
    assert vals[True] == pytest.approx(vals[False], abs=5e-4)


def test_two_level_parametrised_terms_move_with_the_couplings():
    """Coupling-parametrised terms in the two-level family: moving the couplings to c through
    the lifted, split derivative blocks gives the split Hamiltonian whose bond terms are scaled
    to c (checked on a random global state against a dense H built from the scaled terms)."""
    d = W.xxz_triangular(3, 0.5, seed=5, two_level=True)
    R = O.Relaxation(d)
    c = d.params * np.linspace(0.6, 1.4, len(d.params))
    b = W._Builder("xxz_scaled", d.n_sites)
    for t in range(d.n_terms):
        sites, m = d.term(t)
        p = int(d.term_param[t])
        b.add_term(sites, m * (c[p] / d.params[p]))
    b.tops = list(d.tops())
    H = E.dense_H(b.build(real=True, two_level=True))
    hc = O.h_at_params(R, c)
    rho = _random_state(9, 3)
    tot = sum(np.trace(hc[e] @ bf_ptrace(rho, [2] * 9, R.clusters[e])).real for e in hc)
    assert tot == pytest.approx(np.trace(H @ rho).real, abs=1e-10)


# ------------------------------------------------------------------------------------------
# Lipschitz factor Lambda_G of the higher-order smoothed dual (Sec. 4.2.2)
# ------------------------------------------------------------------------------------------
#
# grad Q_beta = B^* rho_beta(h + B nu), with B the linear map from messages to the augmented
# Hamiltonians and rho_beta (beta/2)-Lipschitz (Gibbs-state lemma), so the gradient is
# (beta/2) ||B||^2-Lipschitz and the paper's L = beta Lambda_G / 2 needs ||B||^2 <= Lambda_G.
# ||B||^2 is measured here by power iteration on B^* B, applied as "augmented Hamiltonians of
# the messages alone, then their consistency residuals" -- nothing of the Lambda_G formula.

def _BtB(R, nu):
    return R._grad_from_marginals(R.thetas(nu, with_h=False))


def _norm_B_squared(R, iters=400):
    nu = R.symmetrise(R.draw(0, 1.0))
    lam = 0.0
    for _ in range(iters):
        y = _BtB(R, nu)
        lam = _inner(R, nu, y) / _inner(R, nu, nu)
        s = math.sqrt(_inner(R, y, y))
        nu = {k: v / s for k, v in y.items()}
    return lam


# (family, Lambda_G worked out by hand from m_e = |A(e)| + |D(e)|, Lambda_G = max_{e->f}
# (m_f + m_e D_e / D_f)):
#  * Y_3 chain: a 3-interval has m = 2 (two 2-interval children); an interior 2-interval has two
#    3-interval parents and two sites, m = 4; a site has two parent bonds, m = 2.  Messages
#    3 -> 2: 4 + 2 * 8/4 = 8;  2 -> 1: 2 + 4 * 4/2 = 10.  Lambda = 10.
#  * Y_4 chain: 4 -> 3: 4 + 2 * 2 = 8;  3 -> 2: 4 + 4 * 2 = 12;  2 -> 1: 2 + 4 * 2 = 10.  12.
#  * 2 x 2 plaquettes on a periodic square lattice (L >= 3): plaquette m = 4 (four bonds), bond
#    m = 4 (two plaquettes, two sites), site m = 4 (four bonds).  plaquette -> bond:
#    4 + 4 * 16/4 = 20;  bond -> site: 4 + 4 * 4/2 = 12.  Lambda = 20.
#  * up/down triangles on a periodic triangular lattice: triangle m = 3, bond m = 4 (two
#    triangles, two sites), site m = 6.  triangle -> bond: 4 + 3 * 8/4 = 10;  bond -> site:
#    6 + 4 * 4/2 = 14.  Lambda = 14.
#  * two-level chain, windows of 4: a window has one or two overlap children (m <= 2), an
#    interior overlap has two window parents (m = 2).  window -> overlap: 2 + 2 * 16/8 = 6.
LAMBDA_CASES = [
    ("Y3 chain", lambda: W.interval_chain_gue(10, 3, 0.1, seed=3), 10.0),
    ("Y4 chain", lambda: W.interval_chain_gue(10, 4, 0.1, seed=3), 12.0),
    ("plaquettes", lambda: W.tfim_plaquette_batch([4], [1.0]), 20.0),
    ("XXZ triangles", lambda: W.xxz_triangular(4, 0.5, seed=5), 14.0),
    ("two-level chain", lambda: W.interval_chain_gue(10, 4, 0.1, seed=3, two_level=True), 6.0),
]


@pytest.mark.parametrize("name,maker,lam", LAMBDA_CASES, ids=[c[0] for c in LAMBDA_CASES])
def test_lambda_G_hand_values(name, maker, lam):
    assert O.Relaxation(maker()).Lambda == lam


@pytest.mark.parametrize("name,maker,lam", LAMBDA_CASES, ids=[c[0] for c in LAMBDA_CASES])
def test_lambda_G_bounds_the_norm_of_the_message_map(name, maker, lam):
    """||B||^2 <= Lambda_G (what the Lipschitz lemma needs), and Lambda_G is not loose by more
    than a third: a transposed D_e / D_f, or a dropped term of m_e, falls below ||B||^2."""
    R = O.Relaxation(maker())
    nb2 = _norm_B_squared(R)
    assert nb2 <= R.Lambda * (1 + 1e-9)
    assert nb2 >= 0.75 * R.Lambda


@pytest.mark.parametrize("name,maker,lam", LAMBDA_CASES, ids=[c[0] for c in LAMBDA_CASES])
def test_smoothed_dual_gradient_lipschitz_higher_order(name, maker, lam):
    """||grad Q_b(nu) - grad Q_b(nu')|| <= beta Lambda_G / 2 ||nu - nu'|| (Sec. 4.2.2), on random
    pairs and on a pair displaced along B's leading singular direction."""
    R = O.Relaxation(maker())
    beta = 1.3
    L = R.lipschitz(beta)
    pairs = [(R.draw(50 + s, 0.8), R.draw(60 + s, 0.8)) for s in range(3)]
    v = R.symmetrise(R.draw(1, 1.0))
    for _ in range(200):
        y = _BtB(R, v)
        s = math.sqrt(_inner(R, y, y))
        v = {k: x / s for k, x in y.items()}
    a = R.draw(70, 0.3)
    pairs.append((a, R.axpby(1.0, a, 1e-3, v)))
    for a, b in pairs:
        _, ga = R.grad_beta(a, beta)
        _, gb = R.grad_beta(b, beta)
        dg = R.axpby(1, ga, -1, gb)
        dn = R.axpby(1, a, -1, b)
        assert math.sqrt(_inner(R, dg, dg)) <= L * math.sqrt(_inner(R, dn, dn)) + 1e-12


# ------------------------------------------------------------------------------------------
# the certified value's rounding margin (weak duality in floating point)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("D,cplx", [(8, False), (16, False), (16, True), (64, True)])
def test_certify_margin_covers_rounding_on_an_exact_spectrum(D, cplx):
    """Q(0) - margin <= lambda_min for matrices whose spectrum is known exactly and spans
    +-1e6 (weak duality, Sec. 4.1, under rounding): the eigen-solver's computed lambda_min lies
    above the exact one for a good share of the draws, so a missing margin fails here."""
    rng = np.random.default_rng(100 + D)
    above = 0
    for _ in range(40):
        lam = rng.integers(-10 ** 6, 10 ** 6, D)
        R = O.Relaxation(W.exact_spectrum_problem(lam, cplx))
        q, mg = R.certify(R.zeros())
        exact = float(lam.min())
        above += q[0] > exact
        assert q[0] - mg[0] <= exact
        assert q[0] - mg[0] >= exact - 1e-6 * 1e6   # and the margin stays small
    assert above >= 3


# ------------------------------------------------------------------------------------------
# interval hierarchy on a weakly perturbed separable chain (Thm. 3)
# ------------------------------------------------------------------------------------------

def _solve_smoothed(R, betas, maxiter):
    """Maximise Q_beta over Hermitian messages for each beta in turn (warm started) with
    L-BFGS on the oracle's value and gradient; any messages certify Q(nu) <= f*_t, so this only
    needs to get close to the optimum, not to follow Algorithm 2."""
    from scipy.optimize import minimize
    z = R.zeros()
    keys = sorted(z)
    shapes = {k: z[k].shape for k in keys}

    def unpack(x):
        nu, o = {}, 0
        for k in keys:
            sz = int(np.prod(shapes[k]))
            nu[k] = O.herm(x[o:o + sz].reshape(shapes[k]) + 1j * x[o + sz:o + 2 * sz].reshape(shapes[k]))
            o += 2 * sz
        return nu

    x = np.zeros(sum(2 * int(np.prod(shapes[k])) for k in keys))
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):   # many small eigen-solves: BLAS threads only add contention
        return _lbfgs_stages(R, unpack, keys, x, betas, maxiter, minimize)


def _lbfgs_stages(R, unpack, keys, x, betas, maxiter, minimize):
    for beta in betas:
        def f(x):
            q, g = R.grad_beta(unpack(x), beta)
            return -q[0], -np.concatenate([np.concatenate([g[k].real.ravel(), g[k].imag.ravel()]) for k in keys])
        x = minimize(f, x, jac=True, method="L-BFGS-B",
                     options=dict(maxiter=maxiter, gtol=1e-12, ftol=1e-15)).x
    return unpack(x)


def test_interval_hierarchy_converges_exponentially_on_a_perturbed_separable_chain():
    """H = sum h_i + eps sum v_{i,i+1} with gapped product ground state (Thm. 3): the certified
    (E0 - Q(nu_t))/n, an upper bound on (E0 - f*_t)/n, falls by a large factor with every
    increment of the interval length t and sits far below the product-rounding bound 1/t."""
    n, eps = 8, 0.3
    gaps = []
    E0 = None
    for t in (2, 3, 4):
        d = W.interval_chain_gue(n, t, eps, seed=3, two_level=True)
        if E0 is None:
            E0 = E.ground_energy(d)
        R = O.Relaxation(d)
        nu = _solve_smoothed(R, [2.0 ** s for s in range(0, 16, 3)], 1500)
        q, mg = R.certify(nu)
        gaps.append((E0 - (q[0] - mg[0])) / n)
    assert all(g >= 0 for g in gaps)
    assert gaps[1] <= gaps[0] / 20
    assert gaps[2] <= gaps[1] / 5
    for t, g in zip((2, 3, 4), gaps):
        assert g <= 1e-2 / t


def test_growing_cluster_hierarchy_tightens_the_bound_on_a_torus():
    """Sec. 3.2: C subset C_{+1} gives f*_C <= f*_{C+1} <= E0.  On the periodic 4 x 4 TFIM
    (h = 2.5), C = the 2 x 2 plaquettes, C_{+1} = C with every 2 x 3 and 3 x 2 rectangle (each
    covering two plaquettes): the certified value of the larger family, even from a short solve,
    lies above the converged value of the smaller one and below E0 (Lanczos fixture)."""
    E0 = read_reference_energies()["tfim_torus4x4_h2.5_E0"]
    R0 = O.Relaxation(W.tfim_growing_clusters(4, 2.5, 0))
    R1 = O.Relaxation(W.tfim_growing_clusters(4, 2.5, 1))
    assert all(len(R1.children[e]) == 2 and R1.D[R1.children[e][0]] == 16
               for e in range(R1.n_clusters) if R1.D[e] == 64)
    q0, m0 = R0.certify(_solve_smoothed(R0, [2.0 ** s for s in range(0, 13, 3)], 400))
    q1, m1 = R1.certify(_solve_smoothed(R1, [8.0, 128.0], 120))
    b0, b1 = (q0 - m0)[0], (q1 - m1)[0]
    assert b0 <= E0 and b1 <= E0
    assert b1 >= b0 + 0.03 * 16    # the rectangles tighten the bound by more than 0.03 per site
    # the plaquette family is converged: more iterations move it by far less than that gain
    q0b, m0b = R0.certify(_solve_smoothed(R0, [2.0 ** s for s in range(0, 16, 3)], 800))
    assert abs((q0b - m0b)[0] - b0) <= 0.003 * 16


# ------------------------------------------------------------------------------------------
# spin-1 sites (local dimension 3)
# ------------------------------------------------------------------------------------------

def test_spin1_heisenberg_level1_closed_form():
    """Two spin-1 sites: S.S = (S_tot^2 - 4)/2 has lambda_min = -2 (the singlet), whose one-site
    marginals are 1/3, so singlets on every bond are locally consistent: the level-1 optimum is
    the Anderson bound -2 J (n - 1), reached at zero messages, where the gradient vanishes."""
    n = 6
    R = O.Relaxation(W.spin1_chain(n, J=1.0, Dz=0.0, hx=0.0))
    assert R.Q(R.zeros())[0] == pytest.approx(-2.0 * (n - 1), abs=1e-12)
    _, g = R.grad_beta(R.zeros(), 50.0)
    assert max(float(np.abs(v).max()) for v in g.values()) < 1e-10
    E0 = E.ground_energy(W.spin1_chain(n, J=1.0, Dz=0.0, hx=0.0))
    assert -2.0 * (n - 1) <= E0   # weak duality with the exact ground energy (AKLT-like chain: E0 > -2(n-1))


@pytest.mark.parametrize("maker", [lambda: W.spin1_chain(6, Dz=0.4, hx=0.3),
                                   lambda: W.spin1_chain(6, dm=0.3, top_len=3, subintervals=True),
                                   lambda: W.spin1_chain(7, hx=0.5, top_len=3, two_level=True)])
def test_spin1_weak_duality_random_messages(maker):
    """Q(nu) <= E0 for random messages on spin-1 chains (Sec. 4.1), E0 by Lanczos on 3^n states."""
    d = maker()
    R = O.Relaxation(d)
    E0 = E.ground_energy(d)
    for seed in range(4):
        assert R.Q(R.draw(80 + seed, 0.7))[0] <= E0 + 1e-10
