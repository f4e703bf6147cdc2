"""GPU parity on the paths the kernels take at full size, and on the library's settings:

* slab reuse: with fewer per-workgroup scratch slabs than clusters, every workgroup of the
  large-cluster kernels (workgroup Gibbs kernel, tridiagonal certification, slab Jacobi) handles
  several clusters in turn, as at full size on the 4096-site chain;
* the inverse temperatures the solve reaches (2 Gamma / (n 1e-4) ~ 1e5);
* multi-stage FP32 iterations on 16- and 32-dimensional clusters against the FP64 oracle;
* the certified margin on exactly known spectra and on Jacobi solves stopped early;
* captured graphs after a settings change;
* the autograd wrapper's parameters between forward and backward.

Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import lrh_workloads as W
from oracle import lrh_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_40336_amd import lrh
    lrh.load()


def lrhmod():
    from paper_2609_40336_amd import lrh
    return lrh


def sites_per_instance(desc):
    return np.bincount(desc.site_instance, minlength=desc.n_instances).astype(np.float64)


def max_pair_err(got, want):
    assert set(got) == set(want)
    return max(float(np.abs(got[k] - want[k]).max()) for k in want)


def oracle_marginals(R, marg):
    out = {}
    for D, ids in R.cgroups.items():
        for j, e in enumerate(ids):
            out[R.clusters[e]] = marg[D][j]
    return out


# ------------------------------------------------------------------------------------------
# slab reuse
# ------------------------------------------------------------------------------------------

SLAB_PROBLEMS = {
    # 4 windows of 256 (complex), 5 of 128, 6 of 64, 7 of 32 plus the smaller intervals
    "gue_Y8": lambda: W.interval_chain_gue(11, 8, 0.1, seed=3),
    # two-level windows of 7 sites: 6 windows of 128 over 5 overlaps of 64 (complex)
    "gue_T7_two_level": lambda: W.interval_chain_gue(12, 7, 0.1, seed=4, two_level=True),
    # 2 x 3 plaquettes of a 4 x 4 torus: 16 real 64 x 64 clusters
    "tfim_rect2x3": lambda: W.tfim_rect_plaquettes(4, 1.1),
}


@pytest.mark.parametrize("slabs", [1, 2, 3])
@pytest.mark.parametrize("name", list(SLAB_PROBLEMS))
def test_slab_reuse_matches_oracle(name, slabs):
    """Every large-cluster kernel with fewer slabs than clusters: values 1e-9 per site, entries
    1e-10 (Gibbs at beta = 6 and 300, ground projector, certification), and bit-identical
    results to the default slab count."""
    lrh = lrhmod()
    say(f"[slab reuse] {name} slabs={slabs}")
    d = SLAB_PROBLEMS[name]()
    R = O.Relaxation(d)
    nu_o = R.draw(17, 0.4)
    n = sites_per_instance(d)
    P = lrh.Problem(d, 0)
    Pd = lrh.Problem(d, 0)          # default slab count
    P.set_slab_limit(slabs)
    nu = P.from_dense(R.to_pairs(nu_o))
    for beta in (6.0, 300.0, 0.0):
        q, g, m = P.dual_eval(nu, beta, grad=True, marg=True)
        qd, gd, md = Pd.dual_eval(nu, beta, grad=True, marg=True)
        torch.cuda.synchronize()
        assert torch.equal(q, qd) and torch.equal(g, gd) and torch.equal(m, md)
        if beta > 0:
            q_o, g_o = R.grad_beta(nu_o, beta)
            _, rho = R.gibbs(nu_o, beta)
        else:
            q_o, g_o = R.subgrad(nu_o)
            _, rho = R.ground(nu_o)
        tol = 1e-10 if beta < 10 else max(2e-9, 1e-12 * beta)
        assert np.all(np.abs(q.cpu().numpy() - q_o) <= 1e-9 * n)
        assert max_pair_err(P.to_dense(g), R.to_pairs(g_o)) < tol
        assert max_pair_err(P.marg_dense(m), oracle_marginals(R, rho)) < tol
    q, mg, lm = P.certify(nu, lmin=True)
    qd, mgd, lmd = Pd.certify(nu, lmin=True)
    torch.cuda.synchronize()
    assert torch.equal(q, qd) and torch.equal(mg, mgd) and torch.equal(lm, lmd)
    q_o, mg_o = R.certify(nu_o)
    assert np.all(np.abs(q.cpu().numpy() - q_o) <= 1e-9 * n)
    assert np.all(q.cpu().numpy() - mg.cpu().numpy() <= q_o + 1e-12 * n)
    assert P.check() == (0, 0)


def test_slab_reuse_in_the_accelerated_loop():
    """Graph-replayed FP32 iterations with two slabs equal the default slab count bit for bit
    (the graph is recaptured after the limit changes)."""
    lrh = lrhmod()
    say("[slab reuse] accelerated loop gue_Y8")
    d = SLAB_PROBLEMS["gue_Y8"]()
    out = []
    for slabs in (0, 2):
        P = lrh.Problem(d, 0)
        nu, ze = P.zeros(True), P.zeros(True)
        st = P.new_nesterov_state(4.0)
        P.step_nesterov(nu, ze, st, 64, fused=True)
        P.set_slab_limit(slabs)
        P.step_nesterov(nu, ze, st, 64, fused=True)
        torch.cuda.synchronize()
        out.append(nu.clone())
    assert torch.equal(out[0], out[1])


# ------------------------------------------------------------------------------------------
# Gibbs states at the inverse temperature of the solve
# ------------------------------------------------------------------------------------------

BIG_BETA = {   # default shapes: one-wave exponential at D = 16, 32, workgroup above
    "plaq_batch": lambda: W.tfim_plaquette_batch([3, 4, 5], [0.7, 2.0, 3.5]),
    "gue_Y5": lambda: W.interval_chain_gue(9, 5, 0.1, seed=3),
    "gue_Y8": lambda: W.interval_chain_gue(10, 8, 0.1, seed=3),
    "tfim_rect2x3": lambda: W.tfim_rect_plaquettes(4, 1.1),
}


@pytest.mark.parametrize("beta", [2.5e4, 2e5])
@pytest.mark.parametrize("name", list(BIG_BETA))
def test_gibbs_at_solve_beta_matches_oracle(name, beta):
    """beta up to 2e5 (the solve's 2 Gamma / (n 1e-4) is 1.25e5 on the plaquette sweep and 2e5 on
    the 5-site interval chain): about 21 squarings.  Values 1e-9 per site; entries within the
    exponential's backward error times the Gibbs state's Lipschitz constant beta / 2
    (max(2e-9, 1e-12 beta))."""
    lrh = lrhmod()
    say(f"[gibbs big beta] {name} beta={beta}")
    d = BIG_BETA[name]()
    P = lrh.Problem(d, 0)
    R = O.Relaxation(d)
    nu_o = R.draw(43, 0.5)
    q, g, m = P.dual_eval(P.from_dense(R.to_pairs(nu_o)), beta, grad=True, marg=True)
    torch.cuda.synchronize()
    q_o, g_o = R.grad_beta(nu_o, beta)
    _, rho = R.gibbs(nu_o, beta)
    n = sites_per_instance(d)
    tol = max(2e-9, 1e-12 * beta)
    err_q = float(np.max(np.abs(q.cpu().numpy() - q_o) / n))
    err_g = max_pair_err(P.to_dense(g), R.to_pairs(g_o))
    err_m = max_pair_err(P.marg_dense(m), oracle_marginals(R, rho))
    say(f"  per-site value err {err_q:.2e}, gradient {err_g:.2e}, marginal {err_m:.2e}")
    assert err_q <= 1e-9
    assert err_g < tol and err_m < tol
    assert P.check() == (0, 0)


@pytest.mark.parametrize("name", list(BIG_BETA))
@pytest.mark.parametrize("beta", [1024.0, 12288.0])
def test_fp32_gibbs_at_solve_beta(name, beta):
    """Float messages at the solve's beta (degree-8 polynomial, the squarings after the fourth on
    the FP32 matrix cores, theta assembled in FP32): F_beta per site within 2e-6 of the FP64
    oracle evaluated at the same (float-rounded) messages -- F_beta is 1-Lipschitz in theta, so
    the float assembly and squarings move it by about their backward error, a few u_32 = 6e-8
    times ||theta|| (up to ~30) per cluster; observed at most 2e-7 -- and every marginal a
    density matrix (unit trace, no eigenvalue below -1e-5)."""
    lrh = lrhmod()
    say(f"[fp32 gibbs big beta] {name} beta={beta}")
    d = BIG_BETA[name]()
    P = lrh.Problem(d, 0)
    R = O.Relaxation(d)
    nu32 = P.from_dense(R.to_pairs(R.draw(47, 0.5)), f32=True)
    q, _, m = P.dual_eval(nu32, beta, marg=True)
    torch.cuda.synchronize()
    nu_o = R.from_pairs(P.to_dense(nu32))
    q_o, _ = R.grad_beta(nu_o, beta)
    n = sites_per_instance(d)
    err_q = float(np.max(np.abs(q.cpu().numpy() - q_o) / n))
    say(f"  per-site value err {err_q:.2e}")
    assert err_q <= 2e-6
    for c, rho in P.marg_dense(m).items():
        assert abs(np.trace(rho).real - 1.0) <= 1e-5
        assert np.linalg.eigvalsh(rho).min() >= -1e-5
    assert P.check() == (0, 0)


# ------------------------------------------------------------------------------------------
# multi-stage FP32 iterations on 16- and 32-dimensional clusters
# ------------------------------------------------------------------------------------------

FP32_STAGES = {
    "plaq_batch": lambda: W.tfim_plaquette_batch([3, 4, 5], [0.7, 2.0, 3.5]),
    "gue_Y5": lambda: W.interval_chain_gue(9, 5, 0.1, seed=3),
    "gue_T5_two_level": lambda: W.interval_chain_gue(10, 5, 0.1, seed=3, two_level=True),
}


@pytest.mark.parametrize("name", list(FP32_STAGES))
def test_fp32_fused_stages_certified_vs_fp64_oracle(name):
    """beta = 1 .. 256 doubling, 40 accelerated iterations per stage (each stage restarts from
    the current messages), graph-replayed FP32 iterations certified in FP64, against the FP64
    oracle running the same schedule: certified values within 1e-6 per site."""
    lrh = lrhmod()
    say(f"[fp32 stages] {name}")
    d = FP32_STAGES[name]()
    P = lrh.Problem(d, 0)
    R = O.Relaxation(d)
    sched = [(2.0 ** s, 40) for s in range(9)]
    nu, ze = P.zeros(True), P.zeros(True)
    for beta, K in sched:
        st = P.new_nesterov_state(beta)
        P.step_nesterov(nu, ze, st, K, fused=True)
    q, mg, _ = P.certify(nu)
    torch.cuda.synchronize()
    nu_o = O.nesterov(R, sched)
    q_o, mg_o = R.certify(nu_o)
    n = sites_per_instance(d)
    err = np.abs((q - mg).cpu().numpy() - (q_o - mg_o)) / n
    say(f"  per-site certified difference {err.max():.2e}")
    assert np.all(err <= 1e-6)


# ------------------------------------------------------------------------------------------
# the certified margin
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("D,cplx", [(8, False), (8, True), (16, False), (16, True), (64, True), (128, True),
                                    (256, False), (256, True)])
def test_certify_on_exact_spectra(D, cplx):
    """Terms whose spectrum is known exactly (integers up to 1e6): q - margin <= lambda_min
    exactly, on the Jacobi (D = 8), register-row tridiagonal (D = 16), workgroup tridiagonal
    (D = 64, 128) and Lanczos + Cholesky (D = 256; at 64 and 128 too with method 3) kernels.
    Half the draws separate the lowest eigenvalue from the rest by 2e5, where the certificate
    must hold without falling back; on the others either path may serve."""
    lrh = lrhmod()
    say(f"[certify exact spectrum] D={D} cplx={cplx}")
    rng = np.random.default_rng(300 + D + cplx)
    for t in range(12 if D <= 64 else 6):
        lam = rng.integers(-10 ** 6, 10 ** 6, D)
        gapped = t % 2 == 0
        if gapped:
            lam[int(np.argmin(lam))] = int(lam.min()) - 200000
        d = W.exact_spectrum_problem(lam, cplx)
        P = lrh.Problem(d, 0)
        for method in ((0, 3) if D >= 64 else (0,)):
            P.set_certify_method(method)
            q, mg, _ = P.certify(P.zeros())
            torch.cuda.synchronize()
            exact = float(lam.min())
            assert q.item() - mg.item() <= exact
            assert q.item() - mg.item() >= exact - 1e-6 * 1.2e6
            fb = P.certify_fallbacks()
            if gapped and (D >= 256 or method == 3):
                assert fb == 0


@pytest.mark.parametrize("name", ["xxz_tri3", "randchain_Y3_complex"])
def test_certify_holds_when_jacobi_stops_early(name):
    """A sweep cap of 1 leaves off-diagonal mass in the 8 x 8 Jacobi solves: the margin takes it
    (Weyl), so q - margin stays below the oracle's exact Q.  A loosened iteration tolerance does
    not reach certification at all."""
    lrh = lrhmod()
    say(f"[certify early stop] {name}")
    d = (W.xxz_triangular(3, 0.5, seed=5) if name == "xxz_tri3"
         else W.random_chain(7, seed=2, top_len=3, subintervals=True))
    P = lrh.Problem(d, 0)
    R = O.Relaxation(d)
    nu_o = R.draw(5, 0.6)
    nu = P.from_dense(R.to_pairs(nu_o))
    q_o, mg_o = R.certify(nu_o)
    n = sites_per_instance(d)
    P.set_jacobi(1, 0.0)
    q, mg, _ = P.certify(nu)
    torch.cuda.synchronize()
    b = (q - mg).cpu().numpy()
    assert np.all(b <= q_o)
    assert np.all(mg.cpu().numpy() > mg_o)        # the off-diagonal mass entered the margin
    P.set_jacobi(30, 1e-4)
    q, mg, _ = P.certify(nu)
    torch.cuda.synchronize()
    assert np.all(np.abs(q.cpu().numpy() - q_o) <= 1e-9 * n)
    assert np.all((q - mg).cpu().numpy() <= q_o)


# ------------------------------------------------------------------------------------------
# captured graphs after a settings change
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("change", ["shape", "jacobi"])
def test_graph_recaptured_after_settings_change(change):
    """Run 64 graph-replayed iterations, change a setting that the kernels take as an argument
    (the 16-dimensional clusters' launch shape, or the Jacobi sweep cap of their LDS kernel),
    and run 128 more: equal bit for bit to plain iterations under the same sequence."""
    lrh = lrhmod()
    say(f"[graph after settings] {change}")
    d = W.tfim_plaquette_batch([3, 4], [0.9, 2.1])
    res = []
    for fused in (False, True):
        P = lrh.Problem(d, 0)
        if change == "jacobi":
            P.force_shape(16, 16)
        nu, ze = P.zeros(), P.zeros()
        st = P.new_nesterov_state(2.0)
        P.step_nesterov(nu, ze, st, 64, fused=fused)
        if change == "shape":
            P.force_shape(16, 16)      # matrix-exponential kernel -> LDS Jacobi
        else:
            P.set_jacobi(2, 0.0)       # two sweeps: different (unconverged) iterates
        P.step_nesterov(nu, ze, st, 128, fused=fused)
        torch.cuda.synchronize()
        res.append(nu.clone())
    assert torch.equal(res[0], res[1])


# ------------------------------------------------------------------------------------------
# autograd wrapper: the couplings of the forward pass
# ------------------------------------------------------------------------------------------

def test_smoothed_dual_backward_uses_its_forward_couplings():
    """Two forwards at different couplings, then backward of the first: the gradient is the
    oracle's at the first couplings.  Without parameters the parameter gradient is None."""
    lrh = lrhmod()
    say("[autograd] SmoothedDual couplings")
    d = W.xxz_triangular(3, 0.5, seed=5)
    P = lrh.Problem(d, 0)
    R = O.Relaxation(d)
    nu_o = R.draw(7, 0.3)
    beta = 1.5
    c1 = torch.tensor(d.params * 1.1, dtype=torch.float64, device="cuda", requires_grad=True)
    c2 = torch.tensor(d.params * 0.8, dtype=torch.float64, device="cuda", requires_grad=True)
    nu = P.from_dense(R.to_pairs(nu_o)).requires_grad_(True)
    q1, _ = lrh.smoothed_dual(nu, c1, P, beta)
    q2, _ = lrh.smoothed_dual(nu, c2, P, beta)
    q1.sum().backward()
    nb_o, pb_o = O.dual_vjp(R, nu_o, beta, np.ones(1), None, params=d.params * 1.1)
    assert np.max(np.abs(c1.grad.cpu().numpy() - pb_o)) < 1e-10
    q_o = R.Q_beta(nu_o, beta)   # at the build-time couplings: differs from both
    assert abs(q1.item() - q2.item()) > 1e-3 and abs(q1.item() - q_o[0]) > 1e-3
    # no parameters: the wrapper returns no parameter gradient
    nu2 = P.from_dense(R.to_pairs(nu_o)).requires_grad_(True)
    P.set_params(torch.tensor(d.params, dtype=torch.float64, device="cuda"))
    q3, _ = lrh.smoothed_dual(nu2, None, P, beta)
    q3.sum().backward()
    assert nu2.grad is not None


def test_sustained_fp64_mfma_measurement():
    """The measurement aid behind the roofline reports returns a rate between a tenth of and the
    published dense FP64 peak (78.6 TFLOP/s)."""
    lrh = lrhmod()
    say("[measure] sustained fp64 mfma")
    v = lrh.lrh_measure_fp64_mfma(0)
    say(f"  {v:.1f} TFLOP/s")
    assert 7.86 < v <= 78.6 * 1.02
